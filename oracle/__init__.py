"""FP64 CPU oracle for DIAM with P periodically synchronised chains.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package.  The product
path (``paper_1506_05741_amd``) never imports it and shares no code with it:
the oracle is a plain, slow, obviously correct restatement of the method of
Chen, Keyes, Law and Ltaief, "Accelerated dimension-independent adaptive
Metropolis" (arXiv:1506.05741), in NumPy float64, against which the HIP path
is checked.

Modules
-------
``targets``  log-densities (Gaussian, Bayesian logistic regression, the
             paper's twisted "boomerang" map on d = 2).
``diam``     the sampler: DIAM proposal (Section 2.3.4, eqs. diam / diamnl),
             Metropolis-Hastings acceptance (Section 2.2, eq. accept, in the
             form of Algorithm 1), the moment merge of Section 2.4.1 with
             M = 1, Cholesky with a diagonal-jitter rule, and two-stage
             delayed acceptance with a surrogate.
``psrf``     potential scale reduction factor of the chains (Section 2.4.2).
``ess``      integrated autocorrelation time / effective sample size
             (Section 2.2, eq. mse) via Geyer's initial monotone sequence.
``mlp``      the 512-256-256-1 GELU surrogate, its backward pass and Adam.

Every function is pinned by ``tests/test_oracle_*.py`` against something
other than itself (invariants, closed forms, library routines, quadrature);
see each function's docstring for what pins it.
"""
