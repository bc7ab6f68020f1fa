"""Plain FP64 CPU oracle for the FastDF neutrino push (Elbers, arXiv:2207.14256).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute this package: only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` use it.  It shares no code with the HIP
library (no kernels, headers, tables, constants or helpers); the only things
both sides receive are the seeds and parameters of a workload.

Every function follows one passage of the paper, cited in its docstring by
section and equation label, and is written for clarity, not speed: NumPy
vectorises over particles or modes, FFTs are ``numpy.fft``, quadratures are
``scipy.integrate.quad``.  All arithmetic is float64.

Modules
-------
philox      Philox4x64-10 counter-based generator (Salmon et al. 2011).
background  H(a), conformal-time steps, <eps>(a)             (sec. 3.3, sec. 2).
field       BBKS spectrum, sigma_8, seeded delta_0(k), potentials and
            gradient grids                                    (sec. 2.1, sec. 4).
particles   uniform positions, Fermi-Dirac momenta, pre-initial transform
                                                              (sec. 2.1, eq. transform).
push        CIC interpolation, separable force, KDK leapfrog  (sec. 3.3).
stats       delta-f weights, CIC deposit, binned P(k)          (sec. 2.2, sec. 4).

Pins (what fixes each function independently of itself) live in
``tests/test_oracle_*.py``.  Functions without an independent pin say
"parity unpinned" in their docstring; at present there are none.
"""
