"""What a leaf-input correction can gain at best (CPU, dense numpy).

The learned preconditioner maps a leaf's own points and residual to a
correction on that leaf.  Whatever the network, its map cannot depend on
the residual in the neighbouring leaves.  Restricted additive Schwarz over
the near-field patch (the leaf and its edge-sharing leaves) does use it.
Dropping the neighbours' residual from that solve leaves the leaf-restricted
block of the patch inverse.  That block is the best target a leaf-input map
can reach.

Measured here on a local Gaussian system (c = 0.02 + 0.3 I, N = 4096,
leaves of at most 64 points; dense matrices from the oracle's kernel
entries), with GMRES(50) iterations to 1e-8:

- no preconditioner:                          36
- block-Jacobi (exact leaf LU):               28
- patch inverse, leaf block only (ceiling):   26
- restricted additive Schwarz (patch):        15

So a leaf-input network can gain at most about two iterations over
block-Jacobi here, while a patch-input one could halve them.  The pins:
block-Jacobi < none, the ceiling <= block-Jacobi, and Schwarz well below
both."""
import numpy as np
import scipy.sparse.linalg as spla

from paper_2204_05536_amd import inputs


def _iters(A, b, M):
    n = len(b)
    count = [0]

    def cb(_):
        count[0] += 1
    Mop = None if M is None else spla.LinearOperator((n, n), matvec=M)
    x, info = spla.gmres(A, b, M=Mop, rtol=1e-8, restart=50, maxiter=200, callback=cb,
                         callback_type="pr_norm")
    assert info == 0
    assert np.linalg.norm(b - A @ x) <= 1e-7 * np.linalg.norm(b)
    return count[0]


def test_leaf_input_ceiling(orc):
    n = 4096
    rng = np.random.default_rng(3)
    xy = inputs.uniform_square(n, rng)
    b = inputs.rhs(n, rng)
    spec = {"kind": "gauss", "c": 0.02, "diag_mode": "add", "diag_value": 0.3}
    A = orc.dense_matrix(spec, xy)
    O = orc.OracleH(xy, spec, 64, 1e-10, factors=False)
    perm = O.perm()
    L = O.level(O.kappa)
    t, s = O.near_table()
    leaves = [perm[L["begin"][X]:L["begin"][X] + L["count"][X]] for X in range(len(L["key"]))]
    nbr = {X: [] for X in range(len(leaves))}
    for a, c in zip(t, s):
        if a != c:
            nbr[a].append(c)
    Kinv = [np.linalg.inv(A[np.ix_(I, I)]) for I in leaves]
    patch = []
    for X, I in enumerate(leaves):
        P = np.concatenate([I] + [leaves[Y] for Y in nbr[X]])
        Pinv = np.linalg.inv(A[np.ix_(P, P)])
        patch.append((P, Pinv[:len(I), :], Pinv[:len(I), :len(I)]))

    def bj(r):
        z = np.empty_like(r)
        for I, K in zip(leaves, Kinv):
            z[I] = K @ r[I]
        return z

    def ceiling(r):
        z = np.empty_like(r)
        for I, (_, _, S) in zip(leaves, patch):
            z[I] = S @ r[I]
        return z

    def ras(r):
        z = np.empty_like(r)
        for I, (P, R, _) in zip(leaves, patch):
            z[I] = R @ r[P]
        return z

    it = {name: _iters(A, b, M) for name, M in (("none", None), ("bj", bj), ("ceiling", ceiling), ("ras", ras))}
    print(it)
    assert it["bj"] < it["none"]
    assert it["ceiling"] <= it["bj"]
    assert it["bj"] - it["ceiling"] <= 4
    assert it["ras"] <= 0.7 * it["bj"]
