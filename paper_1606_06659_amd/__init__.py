"""libfbmc: the fully Bayesian MCMC hot path of Landau & Niemi (arXiv 1606.06659) on MI355X.

Submodules:
  fbmc         -- Python binding of the C ABI (include/libfbmc.h)
  build        -- in-tree hipcc build of libfbmc.so for gfx950
  datagen      -- seeded synthetic datasets from the model (inputs only)
  diagnostics  -- R-hat, intervals, ESS and MCSE from moments and traces
"""
