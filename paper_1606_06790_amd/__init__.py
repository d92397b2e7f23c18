"""MI355X (gfx950) hot path of the parallel infinite-size DMRG (arXiv 1606.06790).

* ``lib``     ctypes binding of libidmrg.so: heff_apply, lanczos_solve_batch,
              truncate_twosite, update_env, predict_wavefunction
* ``models``  Heisenberg MPOs with an l-site period, initial blocks (Step 1)
* ``driver``  the parallel iDMRG loop on one GPU (Sec. 3)
* ``build``   compiles libidmrg.so with hipcc for gfx950

Importing the package loads nothing; the library is loaded on first use and
its absence is an error (there is no fallback path).
"""
