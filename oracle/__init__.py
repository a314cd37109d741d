"""CPU FP64 oracle of the IP-GFCC hot path -- TEST INFRASTRUCTURE ONLY.

Plain, slow, obviously-correct NumPy/SciPy implementations written from the paper:
* ``fock``   brute-force Fock-space construction (tiny models) -- the trust anchor;
* ``hbar``   closed-form H-bar blocks; ``sigma`` the IP sigma product, its transpose, b, c;
* ``solve``  dense and GMRES shifted solves, G and A (Eqs. xplin, gfcclineqn, gfxn2);
* ``diis``   the complex DIIS solver of the convergence study (Fig. 3);
* ``mor``    the reduced-order model and its adaptive refinement (Eq. model);
* ``mixed``  FP64 iterative refinement around reduced-precision GMRES;
* ``adjoint`` gradient of windowed spectral weight with respect to orbital energies.

Only ``tests/``, ``__graft_entry__.smoke()`` and ``bench.py``'s cpu_baseline leg may import
this package. It shares no code with the HIP library; both read inputs from ``synth``.
"""
