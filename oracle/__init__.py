"""Reference (oracle) implementation of PSWF fast Ewald summation — TEST INFRASTRUCTURE ONLY.

Plain, slow, float64 CPU code written from the paper (Bostrom, Tornberg, af Klinteberg,
"Fast Ewald summation using prolate spheroidal wave functions", arXiv 2602.16591).
It shares no code with the HIP library in ``paper_2602_16591_amd``: neither package imports
the other. Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package; the product path never does.

Modules
-------
pswf    the first prolate spheroidal wave function psi_0^c (Sec. 2.5, App. B)
params  parameter selection (Alg. 3, Sec. 6) with the rounding rules of the design notes
direct  direct Ewald sums: Fourier-space sum (Alg. 1), real-space residual (Sec. 3.1.1),
        self term (Sec. 3.1), Gaussian Ewald (Example 1), energy and forces (Remark in 3.1)
fast    fast Fourier-space summation (Alg. 2) in float64, step by step in the paper's order
pool    the same steps of ``fast`` over particle chunks in worker processes (no arithmetic of
        its own), for systems of a million particles
"""
