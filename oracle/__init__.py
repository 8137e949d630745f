"""FP64 CPU oracle for the preconditioned Krylov solve of the Grunwald
discretisation of the space-fractional diffusion equation (Barakitis,
Ekstrom, Vassalos, "Preconditioners for Fractional Diffusion Equations Based
on the Spectral Symbol").

TEST INFRASTRUCTURE ONLY.  This package is a plain, slow, obviously correct
restatement of the paper's definitions in NumPy/SciPy float64.  Only the test
suite, the smoke check of the entry module and the CPU-baseline leg of the
benchmark may import it.  The GPU library never imports, links or calls it,
and it shares no code, tables or constants with the GPU library: the only
shared module is ``fde_inputs`` (seeded problem data, no solver arithmetic).

Modules
  grunwald   Grunwald weights g_k (eq. grunwald1) and WSGD weights w_k (Sec. 1.3)
  symbol     generating functions g_a, w_a (Sec. 2.1), symbols p_a, q_a (Thm. 2)
  transforms DST-I matrix S_n (eq. sine_transform), Toeplitz matrices T, S
             (eqs. grunwaldmatrix1/2), Toeplitz products
  system     coefficient matrices M (eq. first_order_1d_coefficient_matrix,
             Sec. 1.4 / eq. coef:2d) and right-hand sides
  precond    P_F (eq. prop_1D, eq. 2D_preconditioner), its constant-coefficient
             forms (Sec. 3.1 Case I, eq. 2D_preconditioner_proof_case) and the
             comparison preconditioners of Table 2
  krylov     FGMRES(m) with CGS2 (build mode), PCG, and the unrestarted
             left-preconditioned GMRES that reproduces Tables 1-4 (paper mode)
  examples   Examples 1-3 of Section 4 (coefficients, sources, exact solutions)

Parity status: every function is pinned by tests under ``tests/`` against
values the paper prints (Tables 1-4), closed forms, dense brute force or
invariants.  The oracle has no mirror of the GPU library's mixed-precision
form (float32 inner GMRES): that form is checked through its float64 true
residual, recomputed here, and against the oracle's float64 solution with
the diagonal-dominance bound ||M^{-1}||_inf <= 1/nu of the first-order scheme.
"""
