"""MI355X-native weighted betweenness centrality (Brandes' method on gfx950).

Submodules:
  bc        -- Python binding of the C ABI (include/bc.h) over libbcgpu.so
  graphgen  -- seeded synthetic graph generators
  build     -- builds libbcgpu.so with hipcc
"""
