"""FP64 CPU oracle for the PDV multiple-scattering Monte Carlo.

TEST INFRASTRUCTURE ONLY.  Only tests/, __graft_entry__.smoke() and the
cpu_baseline leg of bench.py may import, call, link or execute anything in
this package.  The product (paper_2012_00963_amd/ and its HIP library) never
touches it, and the two share no code: no kernels, headers, helpers, tables
or constant generators.

Contents (each function cites the passage of Shi et al., arXiv 2012.00963,
that it follows):
  pdv_oracle.cpp  scalar FP64 transport + tally (Sec. II.B, eq. 4, 7-19), and
                  the paper's literal procedure (fixed-step marching,
                  acceptance-rejection angles; Sec. II.B steps 2-7)
  mc.py           ctypes driver; builds tables with tables.py
  tables.py       layer depths (eq. 8, 20), log-normal quadrature (eq. 21),
                  size-averaged Mie optics (eq. 11-14), integer phase CDF
  mie.py          Mie series (eq. 12, 14)
  stage2.py       heterodyne beat signal (eq. 2-3) and spectrogram (Sec. I)
  ss_model.py     corrected single-scattering spectrum and peak relations
                  (eq. 22-35)

Pins: every function is checked by the CPU tests against closed forms,
invariants, textbook special cases, library routines or the paper's worked
numbers; the whole multiple-scattering walk is checked against the exact
reflection of a deep, isotropically scattering slab (Chandrasekhar's
H-function, tests/hfunc.py).  Parity unpinned: the velocity spectrum of a
general cloud has no independent reference value (beyond that, only its
parts are pinned: free flight, samplers, Doppler telescoping, conservation,
single-scattering and surface-only classes), and the back-scattering
efficiency K_back used by the single-scattering comparator (eq. 25) is a
reading of the paper, not a value it prints.
"""
