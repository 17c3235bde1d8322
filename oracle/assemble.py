"""Patch assembly at known positions with blended overlaps (Sec. 2.5: adjacent
scans keep overlapping regions, which are blended to hide the seams; a field
of view with no neighbour is placed by its scan position).  Registration by
image features is not part of this step: positions are given.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Readings taken (the paper describes the blend only in words):
* every reconstructed tile carries its own constant phase (the KK step fixes
  each tile's DC phase independently), so tiles are first brought to a common
  phase: with C_tu = sum over the overlap of F_t conj(F_u), the phases theta
  maximise sum_tu Re(C_tu exp(-j (theta_t - theta_u))), i.e. exp(j theta) is
  the leading eigenvector of the Hermitian matrix C (angular synchronisation).
  Each connected group of overlapping tiles is synchronised on its own, its
  lowest-numbered tile at phase 0 (a tile with no neighbour keeps phase 0);
* the blend is a normalised weighted sum: canvas(p) = sum_t w_t(p) F_t(p)
  exp(-j theta_t) / sum_t w_t(p), zero where no tile covers p, with the
  separable ramp w(y, x) = ramp(y) ramp(x), ramp(v) = min(1, (v + 1/2) / R,
  (n - v - 1/2) / R) over a tile of side n and ramp width R.
"""

import numpy as np


def overlap_matrix(fields, pos, min_overlap=1):
    """C (T x T, Hermitian) of the tiles' overlap correlations; fields (T, n, n)
    complex, pos (T, 2) integer (y0, x0) canvas offsets."""
    T, n, _ = fields.shape
    C = np.zeros((T, T), complex)
    for t in range(T):
        for u in range(t + 1, T):
            y0 = max(pos[t][0], pos[u][0])
            y1 = min(pos[t][0], pos[u][0]) + n
            x0 = max(pos[t][1], pos[u][1])
            x1 = min(pos[t][1], pos[u][1]) + n
            if y1 - y0 < min_overlap or x1 - x0 < min_overlap:
                continue
            ft = fields[t][y0 - pos[t][0]:y1 - pos[t][0], x0 - pos[t][1]:x1 - pos[t][1]]
            fu = fields[u][y0 - pos[u][0]:y1 - pos[u][0], x0 - pos[u][1]:x1 - pos[u][1]]
            C[t, u] = np.sum(ft * np.conj(fu))
            C[u, t] = np.conj(C[t, u])
    return C


def synchronise_phases(C):
    """theta (T,): per connected group of C's graph, the phases of the leading
    eigenvector of the group's block, rotated so its first tile is at 0."""
    T = C.shape[0]
    theta = np.zeros(T)
    seen = np.zeros(T, bool)
    for s in range(T):
        if seen[s]:
            continue
        group, stack = [], [s]
        seen[s] = True
        while stack:
            t = stack.pop()
            group.append(t)
            for u in np.nonzero(C[t] != 0)[0]:
                if not seen[u]:
                    seen[u] = True
                    stack.append(u)
        group = sorted(group)
        if len(group) == 1:
            continue
        ev, V = np.linalg.eigh(C[np.ix_(group, group)])
        v = V[:, -1]
        theta[group] = np.angle(v * np.exp(-1j * np.angle(v[0])))
    return theta


def ramp(n, width):
    v = np.arange(n) + 0.5
    return np.minimum(1.0, np.minimum(v / width, (n - v) / width))


def blend(fields, pos, theta, shape, width):
    """Normalised ramp-weighted blend of the phase-aligned tiles on a canvas."""
    T, n, _ = fields.shape
    num = np.zeros(shape, complex)
    den = np.zeros(shape)
    r = ramp(n, width)
    w = np.outer(r, r)
    for t in range(T):
        y, x = pos[t]
        num[y:y + n, x:x + n] += w * fields[t] * np.exp(-1j * theta[t])
        den[y:y + n, x:x + n] += w
    out = np.zeros(shape, complex)
    m = den > 0
    out[m] = num[m] / den[m]
    return out
