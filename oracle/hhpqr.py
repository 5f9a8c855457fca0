"""The Householder method for the PQR problem (oracle; test infrastructure only).

Sec. 2.2, eq. (2.4) and Algorithm "HH".  The basis is never stored as
columns: it is the product of unit reflectors

    Q_k = H_0 H_1 ... H_{k-1},   H_i = I - 2 v_i v_i^T,  ||v_i|| = 1,

and its first k columns Q_k [I_k; 0] are the orthonormal basis.  Reflector
v_i is zero in the rows above row i, so H_j leaves e_0 .. e_{j-1} alone and
appending reflectors never changes the columns already in the basis.

One PQR step for a new block X (n x s), in the paper's order:

1. X~ = H_{k-1} ... H_0 X  (Q_k^T X, all k reflectors on all columns);
2. for column i = 0 .. s-1: u = H_{k+i-1} ... H_k X~[:, i] (the reflectors
   made earlier in this step, applied to this column only);
   P[:, i] = u[0:k]; N[0:i, i] = u[k:k+i];
   lambda = ||u[k+i:]||, sigma = -sgn(u[k+i]), N[i, i] = sigma lambda;
   v~ = u[k+i:] - sigma lambda e_1 and v_{k+i} = v~ / ||v~|| (zero above row
   k+i);
3. U = Q_{k+s}[:, k:k+s], i.e. all k+s reflectors applied (last one first)
   to the unit vectors e_k .. e_{k+s-1}.

Readings where the paper is silent or garbled:
* the listing takes the sign from entry k and the norm over rows k:n in
  every column step; the i-th step needs entry k+i and rows k+i:n (the
  text's own definition of v_{k+i}), which is what is done here;
* sgn(0) = +1, so sigma = -1 when the pivot entry is zero;
* a column whose rows k+i: are all zero (lambda = 0) gets the reflector
  v = e_{k+i} and N[i, i] = 0: any unit vector supported on those rows
  keeps the factorisation exact, and this one is the simplest.  (H = I - 2
  e e^T flips the sign of row k+i in the later columns.)

N can have negative diagonal entries (N[i, i] = sigma lambda).  The PQR
solution with a positive diagonal is unique, so (P, D N, U D) with
D = diag(sign N_ii) is the solution of every other method.
"""

import numpy as np


def _apply_reflector(v, Y):
    """Y <- (I - 2 v v^T) Y in place (Y 2-D)."""
    Y -= 2.0 * np.outer(v, v @ Y)


class HouseholderBasis:
    """A basis of R^n held as unit Householder reflectors (n x k, column i
    zero above row i), grown by ``pqr`` one block at a time."""

    def __init__(self, n):
        self.n = int(n)
        self.V = np.zeros((self.n, 0), dtype=np.float64)

    @property
    def k(self):
        return self.V.shape[1]

    def apply_transpose(self, X):
        """Q_k^T X = H_{k-1} ... H_0 X (the full n x n orthogonal factor)."""
        Y = np.array(X, dtype=np.float64, copy=True)
        if Y.ndim == 1:
            Y = Y[:, None]
        for i in range(self.k):
            _apply_reflector(self.V[:, i], Y)
        return Y

    def apply(self, C):
        """Q_k [C; 0] = H_0 ... H_{k-1} [C; 0] for C with at most n rows."""
        C = np.asarray(C, dtype=np.float64)
        if C.ndim == 1:
            C = C[:, None]
        if C.shape[0] > self.n:
            raise ValueError("C has more rows than the space")
        Y = np.zeros((self.n, C.shape[1]), dtype=np.float64)
        Y[:C.shape[0]] = C
        for i in range(self.k - 1, -1, -1):
            _apply_reflector(self.V[:, i], Y)
        return Y

    def explicit(self):
        """The orthonormal basis Q_k [I_k; 0] (n x k)."""
        return self.apply(np.eye(self.k))

    def pqr(self, X):
        """Algorithm "HH": returns (P, N, U) and appends the s new reflectors."""
        X = np.asarray(X, dtype=np.float64)
        n, s = X.shape
        k = self.k
        if n != self.n:
            raise ValueError("X must have n rows")
        if k + s > n:
            raise ValueError("k + s exceeds the dimension")
        Xt = self.apply_transpose(X)
        P = np.zeros((k, s), dtype=np.float64)
        N = np.zeros((s, s), dtype=np.float64)
        new = []
        for i in range(s):
            u = Xt[:, i].copy()
            for v in new:                      # H_{k+i-1} ... H_k, oldest first
                u -= 2.0 * v * (v @ u)
            P[:, i] = u[:k]
            N[:i, i] = u[k:k + i]
            piv = k + i
            lam = np.sqrt(np.dot(u[piv:], u[piv:]))
            v = np.zeros(n, dtype=np.float64)
            if lam == 0.0:
                v[piv] = 1.0
                N[i, i] = 0.0
            else:
                sigma = -1.0 if u[piv] >= 0.0 else 1.0
                N[i, i] = sigma * lam
                vt = u[piv:].copy()
                vt[0] -= sigma * lam
                v[piv:] = vt / np.sqrt(np.dot(vt, vt))
            new.append(v)
        self.V = np.hstack([self.V, np.stack(new, axis=1)])
        E = np.zeros((k + s, s), dtype=np.float64)
        E[k:, :] = np.eye(s)
        U = self.apply(E)
        return P, N, U


def hh_pqr(basis, X):
    """Functional form: one Algorithm "HH" step on ``basis`` (mutated)."""
    return basis.pqr(X)


def hh_with_zero_rows(basis, at, count):
    """A HouseholderBasis whose reflectors (and so whose basis) carry `count`
    zero rows inserted before row `at` (a zero row of every reflector stays
    a zero row of every product of them)."""
    out = HouseholderBasis(basis.n + count)
    out.V = np.vstack([basis.V[:at], np.zeros((count, basis.V.shape[1])), basis.V[at:]])
    return out
