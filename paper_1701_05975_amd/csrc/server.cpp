// server.cpp -- continuous-batching request server (added with the serving form).
