"""Oracle for the two-phase lattice Boltzmann step: plain, slow, FP64, CPU only.

TEST INFRASTRUCTURE. Only tests/, __graft_entry__.smoke() and the CPU-baseline
leg of bench.py may import, call, link or execute anything in this package. It
shares no code with the HIP library (paper_2112_01975_amd) and never imports it.

  thermo.py       equations of state, Maxwell construction, sigma and kappa(W)
  lbm_oracle.c    the full FP64 step (moments, EOS, Korteweg force, correction,
                  product-form equilibria, LBGK, streaming with bounce-back)
  oracle.py       ctypes binding of lbm_oracle.c
  brute.py        a second, independently written vectorised NumPy step used
                  only to pin lbm_oracle.c on tiny grids
"""
