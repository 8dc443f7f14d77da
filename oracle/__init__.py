"""Plain FP64 CPU oracle for the preconditioned iPEPS step.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
link this package; only the tests, the smoke check and the CPU-baseline leg of
the benchmark use it.  It shares no code with the device path: it is written
from the paper (arXiv:2511.09546) and standard tensor-network definitions in
plain PyTorch CPU float64 (einsum, LAPACK SVD/Cholesky), slow and direct.

Modules
-------
ctmrg        double-layer tensor, trace-boundary start, one simultaneous
             four-corner CTMRG iteration with half-system SVD projectors,
             corner spectra and the convergence loop (Sec. III A: the
             environment "gray circles" of the energy network, Eq. (7)).
observables  reduced density matrices and the energy per site (Eqs. (6)-(7)).
gradient     dE/dA by reverse-mode differentiation of the oracle itself, with
             a full-spectrum SVD adjoint (Sec. III A, "backward mode AD";
             Sec. IV A, the unrolled "(3+20)" step configuration).
metric       local metric N_local (Eq. (11)), the regularised preconditioner
             N + delta I (Sec. III B), the CG / direct solves of
             P g' = g (Sec. III C) used to form the preconditioned gradient
             (Eq. (4)).
step         the whole preconditioned step of one evaluation, composed.
lbfgs        L-BFGS with the Hager-Zhang line search and the preconditioner
             as initial inverse Hessian; adaptive delta (Secs. II, III B,
             IV A).
bp           belief-propagation (chi = 1) environment and its metric
             (Sec. III A).
c4v          the C4v-symmetric real ansatz, QR-based CTMRG with one corner
             and one edge, and its K-step gradient (Sec. IV A).
full_metric  the full tangent-space metric (Eq. (10)) applied matrix-free as
             the mixed ket/bra second derivative of the per-site log-norm,
             and the GMRES solve of one cycle (Sec. III C).

Parity status: every function is pinned by the CPU tests in tests/ (closed
forms, brute-force finite lattices, decoupled chains, invariances, finite
differences, solver identities); see the header of each module.
"""
from . import ctmrg, observables, gradient, metric, step  # noqa: F401
