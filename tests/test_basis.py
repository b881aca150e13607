"""Host-side coefficient transforms (per-branch filter lengths, orthogonal
basis fold) against direct evaluation of the model they describe (CPU)."""
import numpy as np

from paper_1612_09001_amd import basis, signals


def _psi(x, p):
    return np.abs(x) ** (p - 1) * x


def _shift(v, k):
    out = np.zeros_like(v)
    out[k:] = v[:v.size - k] if k else v
    return out


def test_per_branch_lengths_equal_direct_sum(orc):
    """Section 2.1 allows L_p != L_q: zero-padded uniform L reproduces the sum
    with each branch's own taps exactly."""
    rng = np.random.default_rng(3)
    mo, Lm, co, Lc = [1, 3, 5], [5, 3, 2], [1, 3], [4, 5]
    x = signals.ofdm_16qam(300, config_id=61).astype(np.complex128)
    mt = [rng.normal(size=n) + 1j * rng.normal(size=n) for n in Lm]
    ct = [rng.normal(size=n) + 1j * rng.normal(size=n) for n in Lc]
    c = 0.1 - 0.2j
    L, h = basis.pad_branch_lengths(mo, Lm, co, Lc, mt, ct, c)
    assert L == 5 and h.size == (3 + 2) * 5 + 1
    z = orc.forward(x.astype(np.complex64), mo, co, L, h)
    ref = np.full(x.size, complex(np.complex64(c)))
    for p, taps in zip(mo, mt):
        for k, t in enumerate(taps.astype(np.complex64)):
            ref = ref + complex(t) * _shift(_psi(x.astype(np.complex64).astype(np.complex128), p), k)
    for q, taps in zip(co, ct):
        for k, t in enumerate(taps.astype(np.complex64)):
            ref = ref + complex(t) * _shift(np.conj(_psi(x.astype(np.complex64).astype(np.complex128), q)), k)
    assert np.max(np.abs(z - ref)) <= 1e-12 * np.max(np.abs(ref))


def test_orthonormal_u_is_orthonormal():
    x = signals.ofdm_16qam(1 << 14, config_id=62).astype(np.complex128)
    orders = [1, 3, 5, 7]
    u = basis.orthonormal_u(x, orders)
    assert np.isrealobj(u) and np.allclose(u, np.triu(u))
    psi = np.stack([sum(u[m, p] * _psi(x, orders[m]) for m in range(len(orders))) for p in range(len(orders))])
    G = psi @ psi.conj().T / x.size
    assert np.max(np.abs(G - np.eye(len(orders)))) <= 1e-9


def test_fold_orthogonal_equals_orthogonal_model(orc):
    """sum_p h'_p psi'_p (main) + sum_q g'_q conj(psi'_q) (conjugate), evaluated
    directly, equals the oracle's monomial model with the folded coefficients."""
    rng = np.random.default_rng(4)
    x = signals.ofdm_16qam(2000, config_id=63).astype(np.complex64)
    xd = x.astype(np.complex128)
    mo = co = [1, 3, 5]
    L = 3
    u = basis.orthonormal_u(xd, mo)
    ho = rng.normal(size=(3, L)) + 1j * rng.normal(size=(3, L))
    go = rng.normal(size=(3, L)) + 1j * rng.normal(size=(3, L))
    hm = basis.fold_orthogonal(u, ho)
    gm = basis.fold_orthogonal(u, go)
    coeffs = np.concatenate([hm.reshape(-1), gm.reshape(-1), [0.0]])
    z = orc.forward(x, mo, co, L, coeffs.astype(np.complex128).astype(np.complex64))
    psio = [sum(u[m, p] * _psi(xd, mo[m]) for m in range(3)) for p in range(3)]
    ref = np.zeros(x.size, complex)
    for p in range(3):
        for k in range(L):
            ref += ho[p, k] * _shift(psio[p], k) + go[p, k] * _shift(np.conj(psio[p]), k)
    # the folded coefficients pass through complex64: relative error ~1e-7
    assert np.linalg.norm(z - ref) / np.linalg.norm(ref) <= 1e-5
