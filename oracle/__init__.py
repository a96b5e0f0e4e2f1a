"""FP64 CPU oracle for the Fourier-Galerkin projected-CG corrosion-fracture path.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import anything from this package.  The
product (``paper_2305_13081_amd``) never imports it, and this package imports
nothing from the product: the two share no code.

Two levels, following the paper (Pundir, Kammer, Angst, arXiv 2305.13081):

* algorithm level -- plain NumPy FP64 versions of the steps the GPU path takes:
  a naive recursive mixed-radix DFT (``fft``), the forward-difference gradient
  symbol of Sec. 2.6, the projection operators of App. A (eq. g-42), the
  constitutive law of Sec. 2.3, the AT2 phase-field operator of Sec. 2.4
  (eq. crack-fft), the transient heterogeneous diffusion operator, textbook CG,
  and the staggered scheme of Alg. 1;
* definition level (``direct``) -- the same discrete problems assembled as
  real-space stencils and solved by a sparse direct solver, with no FFT at all.

Every module states the passage it follows, and the reading it takes where
a passage is ambiguous or garbled.  Functions without an
independent pin say "parity unpinned" in their docstring (none at present).
"""
