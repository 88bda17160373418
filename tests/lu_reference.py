"""NumPy restatement of the library's blocked LU (test helper, not the oracle).

Same blocking as the device code -- 128-column panels, 8/16-column sub-panels,
partial pivoting with ties to the lowest row, interchanges applied as you go --
so the device factors can be compared element by element and the pivot
sequence bit for bit.  Its solves are checked against LAPACK in the tests."""
import numpy as np

NB = 128


def _perm(start, cnt, pivs):
    R = list(range(start, start + cnt))
    lab = list(range(cnt))
    for j, p in enumerate(pivs):
        if p < start + cnt:
            i2 = p - start
        elif p in R[cnt:]:
            i2 = R.index(p, cnt)
        else:
            R.append(p)
            lab.append(len(R) - 1)
            i2 = len(R) - 1
        lab[j], lab[i2] = lab[i2], lab[j]
    return R, [R[l] for l in lab]


def pad(M):
    n = len(M)
    npad = -(-n // NB) * NB
    P = np.eye(npad)
    P[:n, :n] = M
    return P


def factor(A, IB, pairs=False):
    """pairs: the convention of dense factors formed with the panels in pairs
    (a pair's second interchanges also applied to the first panel's L rows;
    panels 2m and 2m+1 for 2m + 2 < n / NB).  The arithmetic here stays one
    update per panel, so values agree with the device's to rounding."""
    A = A.copy()
    n = len(A)
    ip = np.zeros(n, dtype=np.int64)
    for k0 in range(0, n, NB):
        for sp in range(NB // IB):
            c0 = k0 + sp * IB
            a = A[c0:, c0:c0 + IB].copy()
            sw = []
            for j in range(IB):
                c = c0 + j
                p = c + int(np.argmax(np.abs(a[j:, j])))
                if p != c:
                    a[[j, p - c0]] = a[[p - c0, j]]
                ip[c] = p
                sw.append(p)
                if a[j, j] != 0:
                    # multipliers by the reciprocal of the pivot, as the device does
                    # (division only for subnormal pivots)
                    if abs(a[j, j]) >= np.finfo(a.dtype).tiny:
                        a[j + 1:, j] *= 1.0 / a[j, j]
                    else:
                        a[j + 1:, j] /= a[j, j]
                    a[j + 1:, j + 1:] -= np.outer(a[j + 1:, j], a[j, j + 1:])
            A[c0:, c0:c0 + IB] = a
            R, src = _perm(c0, IB, sw)
            other = list(range(k0, c0)) + list(range(c0 + IB, k0 + NB))
            A[np.ix_(R, other)] = A[src][:, other].copy()
            rest = list(range(c0 + IB, k0 + NB))
            if rest:
                U = A[c0:c0 + IB, rest].copy()
                for j in range(1, IB):
                    U[j] -= a[j, :j] @ U[:j]
                A[c0:c0 + IB, rest] = U
                A[c0 + IB:, rest] -= a[IB:, :IB] @ U
        p = k0 // NB
        second = pairs and p % 2 == 1 and k0 + NB < n
        if second:
            R, src = _perm(k0, NB, ip[k0:k0 + NB])
            prev = list(range(k0 - NB, k0))
            A[np.ix_(R, prev)] = A[src][:, prev].copy()
        if k0 + NB < n:
            R, src = _perm(k0, NB, ip[k0:k0 + NB])
            cols = list(range(k0 + NB, n))
            A[np.ix_(R, cols)] = A[src][:, cols].copy()
            X = A[k0:k0 + NB, cols].copy()
            for j in range(1, NB):
                X[j] -= A[k0 + j, k0:k0 + j] @ X[:j]
            A[k0:k0 + NB, cols] = X
            A[k0 + NB:, k0 + NB:] -= A[k0 + NB:, k0:k0 + NB] @ X
    return A, ip


def solve(A, ip, b, pairs=False):
    b = b.copy()
    n = len(A)
    npan = n // NB

    def interchange(k0):
        for j in range(NB):
            q = ip[k0 + j]
            if q != k0 + j:
                b[[k0 + j, q]] = b[[q, k0 + j]]

    for k0 in range(0, n, NB):
        p = k0 // NB
        if pairs and p % 2 == 1 and p + 1 < npan:
            pass                       # applied with the pair's first panel
        else:
            interchange(k0)
            if pairs and p % 2 == 0 and p + 2 < npan:
                interchange(k0 + NB)
        for j in range(NB):
            b[k0 + j] -= A[k0 + j, k0:k0 + j] @ b[k0:k0 + j]
        b[k0 + NB:] -= A[k0 + NB:, k0:k0 + NB] @ b[k0:k0 + NB]
    for k0 in range(n - NB, -1, -NB):
        r = b[k0:k0 + NB] - A[k0:k0 + NB, k0 + NB:] @ b[k0 + NB:]
        for j in range(NB - 1, -1, -1):
            r[j] = (r[j] - A[k0 + j, k0 + j + 1:k0 + NB] @ r[j + 1:]) / A[k0 + j, k0 + j]
        b[k0:k0 + NB] = r
    return b


def factor_static(A):
    """The blocked LU without row interchanges (static pivoting): per 128-column
    panel, the diagonal block's pivots below 2^-20 of its largest entry are
    replaced by that bound with their sign, L21 = A21 U11^-1, U12 = L11^-1 A12,
    A22 -= L21 U12.  Pivots are the identity."""
    A = A.copy()
    n = len(A)
    for k0 in range(0, n, NB):
        k1 = k0 + NB
        tau = max(np.abs(A[k0:k1, k0:k1]).max() * 2.0 ** -20, np.finfo(np.float32).tiny)
        for k in range(k0, k1):
            pv = A[k, k]
            if not abs(pv) >= tau:
                pv = -tau if pv < 0 else tau
                A[k, k] = pv
            A[k + 1:k1, k] /= pv
            A[k + 1:k1, k + 1:k1] -= np.outer(A[k + 1:k1, k], A[k, k + 1:k1])
        if k1 < n:
            U11 = np.triu(A[k0:k1, k0:k1])
            L11 = np.tril(A[k0:k1, k0:k1], -1) + np.eye(NB)
            A[k1:, k0:k1] = np.linalg.solve(U11.T, A[k1:, k0:k1].T).T
            A[k0:k1, k1:] = np.linalg.solve(L11, A[k0:k1, k1:])
            A[k1:, k1:] -= A[k1:, k0:k1] @ A[k0:k1, k1:]
    return A, np.arange(n)
