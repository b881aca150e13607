"""Host-side coefficient transforms for the APH basis (section 2.1, 2.2).

The library's kernels take one filter length L for every branch and the
monomial basis psi_p(x) = |x|^(p-1) x.  Two forms the paper allows map onto
that exactly:

* per-branch filter lengths L_p, L_q (section 2.1): a branch with fewer taps is
  the same filter with zero taps appended, so ``pad_branch_lengths`` builds the
  uniform-L coefficient vector;
* an orthogonal polynomial basis psi'_p(x) = sum_{m <= p} u_{m,p} |x|^(m-1) x
  (section 2.1; its constants u are in a reference the paper does not
  reproduce): sum_p h'_p psi'_p = sum_m (sum_p u_{m,p} h'_p) psi_m, so
  ``fold_orthogonal`` turns orthogonal-basis coefficients into monomial ones,
  per branch and tap.  ``orthonormal_u`` derives one such u by Gram-Schmidt on
  a signal's amplitude moments (the orthonormal basis of that signal), which
  is what makes least squares in the orthogonal basis well conditioned.

Coefficient vectors follow the section 2.2 stacking: for each main order its
taps, then for each conjugate order its taps, then c.
"""
from __future__ import annotations

import numpy as np


def pad_branch_lengths(main_orders, main_L, conj_orders, conj_L, main_taps, conj_taps, c):
    """Uniform-L coefficient vector from per-branch lengths.

    main_L[i] (conj_L[i]) is the length of the filter of main_orders[i]
    (conj_orders[i]); main_taps[i] (conj_taps[i]) its taps.  Returns (L,
    coeffs complex64) with L = the longest filter and zeros after each
    shorter filter's last tap."""
    lens = list(main_L) + list(conj_L)
    if len(main_L) != len(main_orders) or len(conj_L) != len(conj_orders):
        raise ValueError("one length per order")
    if any(int(v) < 1 for v in lens):
        raise ValueError("filter lengths must be >= 1")
    L = max(int(v) for v in lens)
    out = []
    for taps, n in list(zip(main_taps, main_L)) + list(zip(conj_taps, conj_L)):
        t = np.asarray(taps, dtype=np.complex128).reshape(-1)
        if t.size != int(n):
            raise ValueError("expected %d taps, got %d" % (n, t.size))
        out.extend(list(t) + [0.0] * (L - t.size))
    out.append(complex(c))
    return L, np.asarray(out, dtype=np.complex64)


def orthonormal_u(x, orders) -> np.ndarray:
    """u (len(orders) x len(orders), upper triangular) such that
    psi'_p = sum_m u[m, p] |x|^(m-1) x are orthonormal on the samples x:
    (1/N) sum_n psi'_p(x_n) conj(psi'_q(x_n)) = delta_pq.  Gram-Schmidt on the
    monomials in the given (ascending, odd) order, in FP64."""
    x = np.asarray(x, dtype=np.complex128).reshape(-1)
    orders = [int(p) for p in orders]
    s = np.abs(x) ** 2
    phi = np.stack([s ** ((p - 1) // 2) * x for p in orders])      # monomials, rows
    G = (phi @ phi.conj().T) / x.size                               # Gram of the monomials
    # G[m, p] = mean |x|^(m+p): real, so u is real and the same fold serves the
    # conjugate branch (conj(psi'_q(x)) = sum_m u[m, q] conj(phi_m(x)))
    Lc = np.linalg.cholesky(np.real(G))                             # G = Lc Lc^T
    # psi' = Lc^{-1} phi  ->  psi'_p = sum_m (Lc^{-1})[p, m] phi_m, so u[m, p] = (Lc^{-1})[p, m]
    return np.linalg.inv(Lc).T


def fold_orthogonal(u, h_orth) -> np.ndarray:
    """Monomial coefficients of one branch from orthogonal-basis ones:
    h[m, k] = sum_p u[m, p] h_orth[p, k]  (rows: orders, columns: taps)."""
    u = np.asarray(u, dtype=np.complex128)
    h = np.asarray(h_orth, dtype=np.complex128)
    return u @ h
