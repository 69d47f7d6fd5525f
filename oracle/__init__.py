"""CPU oracle for the nonlocal exchange matrix -- TEST INFRASTRUCTURE ONLY.

Plain, slow, obviously correct float64 NumPy code written from the paper
(Betzinger, Friedrich & Bluegel, "Hybrid functionals within the all-electron
FLAPW method: implementation and applications of PBE0", arXiv:1003.0524).

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package. The library (``paper_1003_0524_amd``)
never does, and this package never imports the library: the two share no code.
The only shared module is ``synth`` (seeded input generators, no method
arithmetic).

Modules
-------
vx         -- the exchange matrix as defined by the vector-matrix-vector form
              (Sec. III.C, eq. "vec-mat-vec") with a dense Coulomb matrix, and the
              exchange energy (Sec. II, eq. "HF exchange energy").
brute      -- the same definition as literal nested loops for tiny sizes.
transform  -- the multipole-moment rotation that makes the Coulomb matrix sparse
              (Sec. III.C, the two-function unitary transformation).
chol       -- Cholesky factor of v(q) and V = -sum Y^H Y (exact re-arrangement).
precision  -- input-rounding emulation of the FP32 / split-BF16 product modes.
mlp        -- float64 reference of the small MLP (forward, backward, Adam).
"""
