"""FP64 CPU oracle for Bayesian shear inference (arXiv 2604.22048).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path imports, calls or
links this package; only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may use it.  It shares no code, table or
constant generator with the HIP library: it is a plain, slow restatement of
the paper's definitions in float64 numpy, written so that each function can
be checked against the paper by eye.

Modules
-------
render      k-space stamp definition, pixel log-likelihood (eq. likelihood-pixels)
            and its gradient by forward-mode differentiation of the stamp;
            Appendix C's correlated-noise and multi-exposure likelihood with
            the covariance formed explicitly.
prior       interim prior of eq. interim-prior in sampling coordinates.
philox      Philox4x32-10 counter-based generator, uniforms, Box-Muller normals.
hmc         potential energy, leapfrog, Metropolis test, dual averaging,
            chain initialisation (eq. initialize).
nuts        the No-U-Turn transition (multinomial trajectory sampling, momentum-sum
            U-turn criterion, maximum tree depth) and a NUTS chain with
            dual-averaging warmup (Section 3.3).
diagnostics multi-chain ESS (Geyer initial monotone sequence), R-hat, and the
            time-per-galaxy extrapolation of Section 4.1.
shear       shear response (eq. shear-transform), its Jacobian
            (eq. true-prior-jacobian-shear), true priors, importance weights
            and the Monte-Carlo shear likelihood (eq. likelihood-shear).
bias        multiplicative and additive shear bias by shape-noise cancellation
            with bootstrap errors (Section 3.5, Table 2).

Every function here is pinned by a ``-m "not gpu"`` test against something
other than itself (closed forms, quadrature, brute force, invariants, known
answer vectors); none is "parity unpinned".
"""
