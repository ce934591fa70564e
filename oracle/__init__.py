"""Oracle: a plain, slow, FP64 CPU implementation of the DNN-MG hot path.

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the CPU
baseline leg of the benchmark may import this package.  It shares no code with
the HIP library (``paper_2106_07687_amd``) and never imports it; the only
common dependency is the seeded input generator in ``synthetic``, which holds
none of the method's arithmetic.

Every function cites the passage of the paper it follows (sections, equations,
Algorithm 1, tables).  Readings of passages where the paper is silent or
ambiguous are listed, with the same names (G1..G9, N1..N15), in the project's
design document.

Modules:
    mesh      refinement with curve projection, hierarchy, patches, transfers
    fem       Q1/Q1 local-projection-stabilised Crank-Nicolson residual and
              analytic Jacobian (Sec. 2.1, eqs. varform/varformv/newton)
    solver    Newton with direct solves; additive cell-Vanka, V-cycle, GMRES
    gru       bias-free GRU stack + dense head, BPTT, Adam
    dnnmg     the DNN-MG correction of Algorithm 1 (prolongate, residual,
              patch network, rhs, restrict)
"""
