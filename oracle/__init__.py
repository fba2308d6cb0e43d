"""FP64 CPU oracle for the overlap-operator hot path (Cundy & Lee, "Overlap fermions on GPUs").

TEST INFRASTRUCTURE ONLY.  Nothing in the library may import, call or link this package; only the
test-suite, the smoke check and the benchmark's CPU-baseline leg use it.  It is a plain, slow,
literal NumPy implementation in complex128 of what the paper defines:

* ``wilson``     -- the Wilson-Dirac operator D_W (Sec. 2, eq. 2) and K = gamma5 (D_W - m_W);
* ``chebyshev``  -- coefficients of a Chebyshev approximation of sign(x), the polynomial p(K/lmax)
                    applied by the forward first-kind recurrence, and the deflated sign function
                    of Sec. 2, eq. 3;
* ``deflation``  -- projection Phi^+ psi, correction Phi diag(w) c, classical Gram-Schmidt twice;
* ``overlap``    -- D[mu] = 1/2 (1 + mu + (1 - mu) gamma5 sign(K)) (Sec. 2, eq. 1) and its adjoint;
* ``force``      -- the gauge-link derivative of Re<chi, p(K/lmax) psi> (reverse mode through the
                    forward recurrence) and the D_W link vector-Jacobian product;
* ``eigen``      -- low eigenpairs of K (dense for tiny lattices, ARPACK otherwise);
* ``solver``     -- D[mu] x = b by conjugate gradients on the normal equations, and the dense
                    matrix of D[mu] for tiny lattices.

Array conventions are those of ``latgen``: ``U[mu, a, b, t, z, y, x]`` and
``psi[..., s, c, t, z, y, x]``, periodic boundaries in all four directions, chiral gamma basis.

Parity pins: every function here is checked in ``tests/test_oracle_*.py`` against closed forms,
algebraic identities, dense linear algebra or finite differences.  None is "parity unpinned".
"""
