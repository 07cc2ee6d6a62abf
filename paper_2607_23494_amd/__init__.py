"""MI355X (gfx950) implementation of the in-situ field-window estimator.

Submodules:
  hermes  -- binding of the C ABI (loads libhermes.so; no fallback)
  synth   -- seeded synthetic catalogues and test fields
  serving -- request loop with resident fields and HBM-budget admission
  build   -- in-tree hipcc build of libhermes.so
The package import itself loads nothing, so the input generators can be
used without a GPU.
"""
