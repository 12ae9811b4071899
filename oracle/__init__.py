"""CPU FP64 oracle for the guarded SIMP state solve (test infrastructure only).

This package is the plain, slow, obviously correct reference that the HIP path
is checked against.  It is NOT part of the product: only the test-suite, the
smoke check and the CPU-baseline leg of the benchmark may import it.  It shares
no code with the HIP library (no kernels, headers, tables or constant
generators); both sides are written independently from the paper.

What it computes (citations are to arXiv 2607.26382):

* ``ke``         - hex8 element stiffness (Sec. 3.1, "Discretization and units").
* ``mesh``       - structured cantilever grid, clamped x=0 face, -z edge load.
* ``operator``   - ersatz SIMP law E = rho_min + (1-rho_min) rho^p (Eq. floor_scaling),
                   frozen operator K = sum_e E_e K_e (Eq. frozen_operator),
                   direct solve and the relative residual (Eq. relative_residual).
* ``multigrid``  - 2:1 trilinear transfers, Galerkin coarse operators, damped
                   node-block Jacobi, fixed V-cycle (Tab. solver-config and the
                   fixed linear V-cycle of Sec. 4.5.3 "Fixed-preconditioner control").
* ``fgmres``     - right-preconditioned flexible GMRES with the residual-history
                   semantics of Tab. residual-semantics.
* ``policy``     - probe features, the two-feature rule (Eq. trigger) and the
                   guarded floor ladder (Alg. floor_policy).
* ``features``   - density statistics used by the learned first-floor selector.
* ``mlp``        - forward/backward of the 8-64-64-4 GELU selector network.
* ``stats``      - Wilson score intervals (Sec. 4.3.1 held-out reference test).
* ``fidelity``   - compliance, element energies and the compliance sensitivity
                   of Sec. 3.1, and the raised-floor perturbation metrics of
                   Sec. 4.4.1 / Tab. perturbation.
* ``topopt``     - linear-hat density filter and its adjoint, the smoothed
                   Heaviside projection (Eq. projection) and the optimality-
                   criteria step with volume bisection (Sec. 3.1, Eq.
                   to_problem; Tab. trajectory-settings).
* ``spectrum``   - extreme eigenvalues and condition number of K(rho_min) and
                   the floor screen of Eq. screen (Sec. 4.2).
* ``adaptive``   - the fine-level adaptive correction of the paper's
                   preconditioner (Tab. solver-config): V-cycle, then inner
                   GMRES(20) with node-block Jacobi, kept if it lowers ||r||.

Every function is pinned by tests under ``tests/test_oracle_*.py`` against
facts the paper or mathematics fix (closed forms, invariants, printed values,
library routines on special cases, exact rational evaluation).  Private
helpers (``ke.grad_products_exact``, ``ke.elasticity_D``, ``ke.hadamard8``,
``fgmres._lsq``, ``topopt.filter_weight_sums``, ``policy.first_rung``) are
pinned through the functions built on them.  Among the pins: the screen
against the values printed in Sec. 4.2; the guard's FP64 value and its
rounding bound against exact rational evaluation; FGMRES's breakdown exit in
an invariant subspace and its non-finite exits; the reference label and the
selector's feature layout by scripted cases; Adam by its closed forms.  A
function without such a pin would say "parity unpinned" here; none does.

Reading of Eq. relative_residual where the paper leaves it undefined: for
f = 0, eta = 0 when r = 0 too (u = 0 solves it exactly); any other f whose
norm is not a finite positive number gives NaN, which no acceptance passes.
"""
