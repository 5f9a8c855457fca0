"""TreeTSPQR with the locally orthogonal basis (oracle; test infrastructure).

Sec. 4.1.  The basis Q (n x k) is never stored explicitly.  It is the
product of a block-diagonal matrix of local orthonormal leaf bases and the
stacked reduction factors:

    Q = blockdiag(Q_1, ..., Q_p) [R_1; ...; R_p],

where the stacked [R_1; ...; R_p] is itself orthonormal because Q is
(the short proof in Sec. 4.1: R^T blockdiag(Q_i)^T blockdiag(Q_i) R = Q^T Q).

One step solves the PQR problem, eq. (1.1), for a new block X:

1. every leaf solves its local problem [Q_i X_i] = [Q_i U_i][[I, P_i],
   [0, N_i]] with the *local subalgorithm*;
2. the reduction step solves the PQR problem on the stacked coefficient
   blocks [[R_i, P_i], [0, N_i]]_i with the *reduction subalgorithm*; it
   yields the global P and N and per-leaf blocks P~_i, N~_i;
3. the leaf factors grow to R_i' = [[R_i, P~_i], [0, N~_i]] and the local
   bases to [Q_i U_i]; the explicit new block is U|_i = [Q_i U_i][P~_i; N~_i].

Recursion (Sec. 4.1, "applied recursively"): the reduction problem is itself
a PQR problem on an orthonormal matrix, so it can be solved by TreeTSPQR
again.  ``fan_in`` builds that recursion: level-1 nodes group ``fan_in``
consecutive leaves, level-2 nodes group ``fan_in`` level-1 nodes, and so on
up to a single root.  ``fan_in=None`` (or >= number of leaves) is the
single-level tree.  Every node stores one k x k block per child; the
composition is Q = B_0 B_1 ... B_L with B_0 = blockdiag(Q_i) and B_l the
block-diagonal matrix of level-l node factors.

Readings adopted where the paper is silent:
* leaf partition: p = max(1, n // leaf_rows) leaves of leaf_rows rows, the
  last leaf takes the remainder (so every leaf has >= leaf_rows rows);
* a local problem needs at least k+s rows for full rank; the class refuses a
  step that would break that;
* the first step (k = 0) is the same procedure with an empty basis: it is the
  TSQR of the start block (Sec. 4.1, tree TSQR);
* Householder as the reduction subalgorithm (the stability table of Sec. 6.1
  uses one method at every level): every reduction node holds its basis as
  unit reflectors over its stacked rows (Algorithm "HH", Sec. 2.2); every
  step inserts s zero rows into them after each child's k rows, the rows of
  that child's new coordinates, as the stacked factors are extended with
  zero rows; the pivots are the node's leading rows (its first child's).
  The diagonal of N then carries the Householder signs and the new basis
  columns the same signs, as with Householder leaves.
"""

import numpy as np

from .hhpqr import HouseholderBasis, hh_with_zero_rows
from .deflate import deflating_pip, deflating_pip_plus
from .pqr import SUBALGORITHMS

DEFLATING = {"pip": deflating_pip, "pip+": deflating_pip_plus}


def leaf_bounds(n, leaf_rows):
    """Row ranges [(r0, r1), ...] of the leaves: the last one takes the rest."""
    if leaf_rows <= 0:
        raise ValueError("leaf_rows must be positive")
    p = max(1, n // leaf_rows)
    bounds = [(i * leaf_rows, (i + 1) * leaf_rows) for i in range(p)]
    bounds[-1] = (bounds[-1][0], n)
    return bounds


def _groups(count, fan_in):
    """Consecutive groups of ``fan_in`` units: [(u0, u1), ...]."""
    if fan_in is None or fan_in >= count:
        return [(0, count)]
    return [(g, min(g + fan_in, count)) for g in range(0, count, fan_in)]


class TreeTSPQR:
    """Stateful TreeTSPQR solver; the basis lives in locally orthogonal form.

    Parameters
    ----------
    n, s        rows and block width
    leaf_rows   leaf height (see ``leaf_bounds``)
    local, reduction
                subalgorithm names from ``oracle.pqr.SUBALGORITHMS``
                ("pip" = BCGS-PIP, "pip+" = BCGS-PIP+, "ref" = the unique
                reference solution); ``local`` may also be "hh": the
                Householder method (Sec. 2.2), each leaf basis then held as
                reflectors (``oracle.hhpqr.HouseholderBasis``);
                ``reduction`` may be "hh" (every reduction node's basis held
                as reflectors).
    fan_in      None for the single-level tree, else the tree fan-in.
    deflate     None, or the relative tolerance delta of the deflating
                reduction (``oracle.deflate``, Sec. 3.1): the single
                reduction node drops the directions whose residual singular
                value is at most delta ||X||_F.  ``last_rank`` is the rank t
                of the latest block; the width stays s (zero columns).
    """

    def __init__(self, n, s, leaf_rows, local="pip+", reduction="pip+", fan_in=None, deflate=None):
        self.n, self.s = int(n), int(s)
        self.bounds = leaf_bounds(self.n, int(leaf_rows))
        self.householder = local == "hh"
        self.local = None if self.householder else SUBALGORITHMS[local]
        self.hh_reduction = reduction == "hh"
        self.reduction = None if self.hh_reduction else SUBALGORITHMS[reduction]
        self.deflate = deflate
        self.last_rank = None
        if deflate is not None:
            if self.hh_reduction or reduction not in DEFLATING or not deflate > 0.0:
                raise ValueError("deflation needs reduction 'pip' or 'pip+' and delta > 0")
            self.reduction = DEFLATING[reduction]
        self.k = 0
        p = len(self.bounds)
        if self.householder:
            self.leaves = [HouseholderBasis(r1 - r0) for (r0, r1) in self.bounds]
        else:
            self.leaves = [np.zeros((r1 - r0, 0)) for (r0, r1) in self.bounds]
        # levels[l] = list of nodes; node = {"children": (c0, c1), "S": [k x k blocks]}
        self.levels = []
        count = p
        while True:
            groups = _groups(count, fan_in)
            self.levels.append([{"children": g, "S": [np.zeros((0, 0)) for _ in range(g[1] - g[0])]}
                                for g in groups])
            count = len(groups)
            if count == 1:
                break
        if deflate is not None and len(self.levels) != 1:
            raise ValueError("deflation is defined for the single-level tree")
        if self.hh_reduction:
            for nodes in self.levels:
                for node in nodes:
                    node["H"] = None      # the node's reflectors (reduction "hh")

    @property
    def p(self):
        return len(self.bounds)

    def step(self, X):
        """Solve the PQR problem for X (n x s); returns (P, N, U) and grows the basis."""
        X = np.asarray(X, dtype=np.float64)
        n, s, k = self.n, self.s, self.k
        if X.shape != (n, s):
            raise ValueError(f"X must be {n} x {s}")
        min_rows = min(r1 - r0 for (r0, r1) in self.bounds)
        if k + s > min_rows:
            raise ValueError("local problem would be rank deficient: k+s > leaf rows")
        # 1. local problems (independent)
        Y = []        # per-unit coefficient blocks [P_i; N_i], (k+s) x s
        locals_ = []
        for i, (r0, r1) in enumerate(self.bounds):
            if self.householder:
                Pi, Ni, Ui = self.leaves[i].pqr(X[r0:r1])     # appends the reflectors
            else:
                Pi, Ni, Ui = self.local(self.leaves[i], X[r0:r1])
            locals_.append(Ui)
            Y.append(np.vstack([Pi, Ni]))
        # 2. reduction, level by level; keep each node's new columns
        new_cols = []
        for nodes in self.levels:
            Y_up = []
            cols_level = []
            for node in nodes:
                c0, c1 = node["children"]
                # stacked basis of the node problem: child block S_c over its
                # old k coordinates, zero rows over the child's s new ones
                B = np.vstack([np.vstack([Sc, np.zeros((s, k))]) for Sc in node["S"]])
                Yv = np.vstack(Y[c0:c1])
                if self.hh_reduction:
                    Pv, Nv, Uv = self._hh_reduce(node, c1 - c0, Yv)
                elif self.deflate is None:
                    Pv, Nv, Uv = self.reduction(B, Yv)
                else:
                    Pv, Nv, Uv, self.last_rank = self.reduction(B, Yv, self.deflate)
                cols_level.append(Uv)
                Y_up.append(np.vstack([Pv, Nv]))
            new_cols.append(cols_level)
            Y = Y_up
        P = Y[0][:k]
        N = Y[0][k:]
        # 3. grow the node factors: S_c' = [[S_c, P~_c], [0, N~_c]]
        for nodes, cols_level in zip(self.levels, new_cols):
            for node, Uv in zip(nodes, cols_level):
                grown = []
                for j, Sc in enumerate(node["S"]):
                    blk = Uv[j * (k + s):(j + 1) * (k + s)]
                    top = np.hstack([Sc, blk[:k]])
                    bot = np.hstack([np.zeros((s, k)), blk[k:]])
                    grown.append(np.vstack([top, bot]))
                node["S"] = grown
        if not self.householder:
            for i in range(self.p):
                self.leaves[i] = np.hstack([self.leaves[i], locals_[i]])
        self.k = k + s
        U = self.apply_Q(np.vstack([np.zeros((k, s)), np.eye(s)]))
        return P, N, U

    def _hh_reduce(self, node, children, Yv):
        """A node's reduction problem by Algorithm "HH" on its reflectors:
        s zero rows inserted after every child's k rows, then one pqr."""
        k, s = self.k, self.s
        if node["H"] is None:
            node["H"] = HouseholderBasis(children * s)
        else:
            for c in range(children - 1, -1, -1):
                node["H"] = hh_with_zero_rows(node["H"], c * k + k, s)
        return node["H"].pqr(Yv)

    @property
    def root_hh(self):
        """The single root's reflectors (reduction "hh")."""
        return self.levels[-1][0]["H"]

    def apply_Q(self, C):
        """Y = Q C for C ((current k) x m): down-sweep of C, then leaf products.

        The product QC of Sec. 5.1 ("second stage"): at every node the child
        coefficient block is S_{v,c} C_v, at the leaves Y_i = Q_i C_i.
        """
        C = np.asarray(C, dtype=np.float64)
        if C.ndim != 2 or C.shape[0] != self.k:
            raise ValueError("C must have k rows")
        coeff = [C]
        for nodes in reversed(self.levels):
            nxt = []
            for node, Cv in zip(nodes, coeff):
                for Sc in node["S"]:
                    nxt.append(Sc @ Cv)
            coeff = nxt
        if self.householder:
            return np.vstack([B.apply(Ci) for B, Ci in zip(self.leaves, coeff)])
        return np.vstack([Qi @ Ci for Qi, Ci in zip(self.leaves, coeff)])

    def explicit_Q(self):
        """The explicit n x k basis (for metrics only)."""
        return self.apply_Q(np.eye(self.k))

    def stacked_factor(self, level=0):
        """Stacked node factors of one level as a matrix (single-level: [R_1;...;R_p])."""
        return np.vstack([Sc for node in self.levels[level] for Sc in node["S"]])
