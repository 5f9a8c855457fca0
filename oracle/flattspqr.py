"""FlatTSPQR (oracle; test infrastructure only).

Sec. 4.2, the flat variant of TSQR applied to the PQR problem, eq. (1.1),
and Algorithm "FlatTSPQR".  The rows are cut into consecutive blocks
X_1, ..., X_p (the same rule as TreeTSPQR's leaves: p = max(1, n // rows),
the last block takes the remainder).  The basis is held as the chain

    Q = [[F_1, 0], [0, I]] [[F_2, 0], [0, I]] ... F_p,

where F_1 (m_1 x k) spans block 1's rows and every later F_i
((k + m_i) x k) spans the k coordinates the chain has reached so far
followed by block i's m_i rows; every F_i has orthonormal columns.  One
step for a new block X solves, in order,

    [F_1 X_1] = [F_1 U_1] [[I, P_1], [0, N_1]],
    [F_i^ext [P_{i-1}; N_{i-1}; X_i]] = [F_i^ext U_i] [[I, P_i], [0, N_i]],

i = 2 .. p, with the local subalgorithm, and returns P = P_p, N = N_p.  The
factors grow to F_1 <- [F_1 U_1] and F_i <- [F_i^ext U_i].  The explicit new
block is U = Q_{k+s} [0; I_s], formed through the chain (the products of
eq. (flattspqr_q)).

Readings adopted where the paper is silent:
* the printed problem for i >= 2 stacks P_{i-1}, N_{i-1} and X_i beside a
  Q_i that spans all three row blocks; Q_i has no rows for N_{i-1}'s s new
  coordinates, so it is taken with s zero rows inserted there
  (F_i^ext = [F_i[:k]; 0; F_i[k:]]), as the tree's reduction step extends its
  factors (Sec. 4.1);
* the first step (k = 0) is the same procedure with empty factors: the flat
  TSQR of the start block;
* with Householder local problems (Sec. 2.2) every F_i is held as unit
  reflectors; inserting zero rows into the reflectors inserts them into the
  basis.  The diagonal of N then carries the Householder signs, as the
  paper's Algorithm "HH" returns it; (P, N D, U D) with D = diag(sign N_ii)
  is the unique positive-diagonal solution.
"""

import numpy as np

from .hhpqr import HouseholderBasis, hh_with_zero_rows
from .pqr import SUBALGORITHMS
from .tspqr import leaf_bounds


def _insert_zero_rows(B, at, count):
    """B with `count` zero rows inserted before row `at` (B 2-D)."""
    return np.vstack([B[:at], np.zeros((count, B.shape[1])), B[at:]])


def _hh_insert_zero_rows(basis, at, count):
    """A HouseholderBasis whose reflectors (and so whose basis) carry `count`
    zero rows before row `at`."""
    return hh_with_zero_rows(basis, at, count)


class FlatTSPQR:
    """Stateful FlatTSPQR solver; the basis lives as the chain of factors.

    Parameters
    ----------
    n, s        rows and block width
    block_rows  height of the row blocks (see ``tspqr.leaf_bounds``)
    local       subalgorithm of the local problems: a name from
                ``oracle.pqr.SUBALGORITHMS`` ("pip", "pip+", "ref") or "hh"
                (Algorithm "HH", the factors held as reflectors)
    """

    def __init__(self, n, s, block_rows, local="pip+"):
        self.n, self.s = int(n), int(s)
        self.bounds = leaf_bounds(self.n, int(block_rows))
        self.householder = local == "hh"
        self.local = None if self.householder else SUBALGORITHMS[local]
        self.k = 0
        if self.householder:
            self.factors = [HouseholderBasis(r1 - r0) for (r0, r1) in self.bounds]
        else:
            self.factors = [np.zeros((r1 - r0, 0)) for (r0, r1) in self.bounds]

    @property
    def p(self):
        return len(self.bounds)

    def _solve(self, i, B, Y):
        """Local PQR problem of block i on the (extended) factor B."""
        if self.householder:
            P, N, U = B.pqr(Y)                   # appends the s reflectors to B
            self.factors[i] = B
        else:
            P, N, U = self.local(B, Y)
            self.factors[i] = np.hstack([B, U])
        return P, N

    def step(self, X):
        """Solve the PQR problem for X (n x s); returns (P, N, U) and grows the basis."""
        X = np.asarray(X, dtype=np.float64)
        n, s, k = self.n, self.s, self.k
        if X.shape != (n, s):
            raise ValueError(f"X must be {n} x {s}")
        r0, r1 = self.bounds[0]
        if k + s > r1 - r0:
            raise ValueError("the first block's problem would be rank deficient: k+s > its rows")
        P, N = self._solve(0, self.factors[0], X[r0:r1])
        for i in range(1, self.p):
            r0, r1 = self.bounds[i]
            F = self.factors[i]
            B = _hh_insert_zero_rows(F, k, s) if self.householder else _insert_zero_rows(F, k, s)
            Y = np.vstack([P, N, X[r0:r1]])
            P, N = self._solve(i, B, Y)
        self.k = k + s
        E = np.vstack([np.zeros((k, s)), np.eye(s)])
        U = self.apply_Q(E)
        return P, N, U

    def _factor_apply(self, i, C):
        F = self.factors[i]
        return F.apply(C) if self.householder else F @ C

    def apply_Q(self, C):
        """Y = Q C for C ((current k) x m), right to left through the chain."""
        C = np.asarray(C, dtype=np.float64)
        if C.ndim != 2 or C.shape[0] != self.k:
            raise ValueError("C must have k rows")
        k = self.k
        Z = self._factor_apply(self.p - 1, C)
        for i in range(self.p - 2, -1, -1):
            Z = np.vstack([self._factor_apply(i, Z[:k]), Z[k:]])
        return Z

    def explicit_Q(self):
        """The explicit n x k basis (for metrics only)."""
        return self.apply_Q(np.eye(self.k))

    def factor(self, i):
        """Block i's factor as an explicit matrix (orthonormal columns)."""
        F = self.factors[i]
        return F.explicit() if self.householder else F
