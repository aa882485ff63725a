"""FP64 CPU oracle for the particle-mesh COLA time step of L-PICOLA (Howlett, Manera & Percival, 2015).

TEST INFRASTRUCTURE ONLY. This package is the slow, plain reference that the GPU library is checked against. Only
``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of ``bench.py`` may import it. The product path
(``paper_1506_03737_amd``, ``liblpc.so``) never imports, links or calls anything in here, and this package imports
nothing from the product path.

Everything is NumPy/SciPy in float64 unless a step is integer by definition (the fixed-point cloud-in-cell deposit).
Each module cites the passage of the paper (section and equation) that it follows. Where the paper is silent or
garbled, the reading taken is stated in the function's docstring.

Modules:
  cosmology  -- expansion rate, growth factors D1/D2 and their derivatives, kick/drift factors (Sec. 2.1, 2.3)
  rng        -- the counter-based SplitMix64 + Box-Muller white noise used by the initial conditions
  ic         -- BBKS linear spectrum, sigma8 normalisation, 2LPT displacements on the particle lattice (Sec. 2.1, 5)
  pm         -- fixed-point CIC deposit, FFT Poisson solve with CIC deconvolution, gradient, CIC gather (Sec. 2.4)
  cola       -- the kick-drift-kick COLA integrator about the stored 2LPT displacements (Sec. 2.2, 2.3)
  spectrum   -- binned power spectrum of a periodic box (Sec. 7.1)
  dft        -- brute-force discrete Fourier transform, used only to pin the FFT-based steps
  net        -- the learned displacement correction: a 3-level 3-D U-Net, its backpropagation and Adam
  bispectrum -- reduced bispectrum Q(k1, k2, k3) with the FFT shell estimator and a brute-force triangle sum (Sec. 7)

Parity status: every function here is pinned by a ``-m "not gpu"`` test against a closed form, an invariant or brute
force, except the BBKS transfer-function constants (parity unpinned: retyped from Bardeen et al. 1986, no printed
value to check them against).
"""
