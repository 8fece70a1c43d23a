"""MI355X (gfx950) parallel-tempering simulation of the +-J Edwards-Anderson
spin glass: checkerboard Metropolis sweeps, replica exchange and Houdayer
cluster moves for many disorder samples at once (Kumar, Gross, Janke, Weigel,
arXiv:2003.04621).

Modules:
  pt         -- ctypes binding of the C ABI (include/pt.h), libptsg.so
  build      -- hipcc build of libptsg.so
  workloads  -- seeded couplings, temperature ladders, named workloads
"""
__all__ = ["pt", "build", "workloads"]
