"""Float64 CPU oracle of the bispectrum-multipole estimator (test infrastructure).

Only ``tests/``, ``__graft_entry__.smoke`` and the CPU-baseline leg of
``bench.py`` may import this package.  It shares no code with the HIP path;
the two meet only through the seeded inputs of ``synth``.

Modules:
  geometry  -- rings, sides, N_tri (Eq. 10), combinations, (k1, mu, t), p, Y weights, bins
  ylm       -- Y_l^m from the explicit Legendre sum (Condon-Shortley phase)
  estimator -- Eq. 6 (brute force), Eqs. 8-9 (FFT), Eq. 13 (second-level binning)
  analytic  -- Eqs. 15, 17, the discrete prediction and Eq. 4 by quadrature
"""
