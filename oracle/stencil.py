"""The interior conservative stencil written out with array slices (oracle;
test infrastructure only).

For a box whose faces are all Dirichlet, every unknown row of Ltilde is the
standard second-order conservative stencil of the Cartesian specialisation of
Sec. 4.1 (the Dirichlet values entering it are zero):
  u_a-row:  sum_b D+_b(kbar D-_b u_a) + sum_{b != a} [D0_a(lam D0_b u_b) + D0_b(mu D0_a u_b)]
with k = lam + 2 mu when b = a and k = mu otherwise, bars two-point means.
This is the same operator as operator.Operator for such boxes (pinned by a
test against the energy assembly), but it needs no sparse matrix, so it
reaches the largest grids (one application at 257^3 nodes takes seconds).
"""

import numpy as np


def ltilde_dirichlet(h, lam, mu, u):
    """Ltilde u at interior nodes (zeros on the faces).  u: (d, *node_shape)
    with zero face values; h: spacings (x, y[, z]); lam, mu: node arrays."""
    d = u.shape[0]
    out = np.zeros_like(u)
    inner = (slice(1, -1),) * d

    def sh(a, axis, s):
        # values at offset s along coordinate axis (NumPy axis d-1-axis), restricted to the interior
        idx = [slice(1, -1)] * d
        k = d - 1 - axis
        n = a.shape[k]
        idx[k] = slice(1 + s, n - 1 + s)
        return a[tuple(idx)]

    def sh2(a, ax1, s1, ax2, s2):
        idx = [slice(1, -1)] * d
        for ax, s in ((ax1, s1), (ax2, s2)):
            k = d - 1 - ax
            n = a.shape[k]
            idx[k] = slice(1 + s, n - 1 + s)
        return a[tuple(idx)]

    A = lam + 2.0 * mu
    for c in range(d):
        uc = u[c]
        acc = np.zeros(uc[inner].shape)
        for b in range(d):
            k = A if b == c else mu
            kp = 0.5 * (sh(k, b, 1) + k[inner])
            km = 0.5 * (k[inner] + sh(k, b, -1))
            acc += (kp * (sh(uc, b, 1) - uc[inner]) - km * (uc[inner] - sh(uc, b, -1))) / h[b] ** 2
        for b in range(d):
            if b == c:
                continue
            ub = u[b]
            # D0_c(lam D0_b u_b)
            t1 = (sh(lam, c, 1) * (sh2(ub, c, 1, b, 1) - sh2(ub, c, 1, b, -1))
                  - sh(lam, c, -1) * (sh2(ub, c, -1, b, 1) - sh2(ub, c, -1, b, -1))) / (4 * h[c] * h[b])
            # D0_b(mu D0_c u_b)
            t2 = (sh(mu, b, 1) * (sh2(ub, b, 1, c, 1) - sh2(ub, b, 1, c, -1))
                  - sh(mu, b, -1) * (sh2(ub, b, -1, c, 1) - sh2(ub, b, -1, c, -1))) / (4 * h[c] * h[b])
            acc += t1 + t2
        out[(c,) + inner] = acc
    return out
