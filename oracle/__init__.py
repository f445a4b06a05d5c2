"""FP64 CPU oracle for the batched HMM micro-problem solve.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import, call or link anything under
``oracle/``.  The product path (``paper_2108_09463_amd``) never does, and the
oracle never imports the product path: the two share only the seeded input
definitions in ``paper_2108_09463_amd.inputs``.

The oracle is plain and slow on purpose.  Every step follows the paper
(Leitenmaier & Runborg, "Heterogeneous multiscale methods for the
Landau-Lifshitz equation"):

* micro problem, eq. (micro) in Section 2.2: the LL equation with exchange
  field H = div(a^eps grad m) solved on [-mu', mu']^d x [0, eta];
* spatial discretization: second-order central differences (Section 2.3,
  Section 4 opening); an optional fourth-order conservative stencil;
* HeunP / RK4P projection time stepping (Section 3.1);
* stability rule dt / dx^2 <= C_stab (Section 3.2, eq. (Cstab));
* averaging kernels K in K^{p,q}, K0 in K_0^{p,q} (Definition 2.3) and the
  upscaling integral, eq. (upscaling);
* normalized interpolation Q_[2k] for micro initial data (Section 4.1, eq. (Q_k));
* macro time stepping MPEA (Section 3.1, eqs. (mpe_update), (h_mpea)).

Readings of passages where the paper is silent or inconsistent are listed in
the module docstrings where they are used.

Parity pins: every function here is pinned by ``-m "not gpu"`` tests against
closed forms, brute force, convergence orders, invariants or values printed in
the paper (tests/test_oracle_*.py).
"""
