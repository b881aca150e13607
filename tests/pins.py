"""Pins of the FP64 oracle to facts fixed by the paper and by mathematics.

Each ``pin_*`` function takes an ``oracle.Oracle`` and raises ``AssertionError``
when the oracle disagrees with the fact it checks.  They run against the real
oracle in ``test_oracle_pins.py`` and against deliberately broken copies of it in
``test_oracle_mutants.py`` (every planted mistake must trip at least one pin).

None of these re-types the oracle's loops: each compares against a different
route -- the Toeplitz basis matrix of Eq. (2), a closed form, an invariant of
Eq. (1), the paper's printed PA coefficients (Eq. 3), finite differences, or
PyTorch autograd.
"""
from __future__ import annotations

import os

import numpy as np

import oracle.brute as brute

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _rng(seed):
    return np.random.default_rng(seed)


def _cx(g, n, scale=1.0):
    return (g.standard_normal(n) + 1j * g.standard_normal(n)) * (scale / np.sqrt(2.0))


def _coeffs(g, main, conj, L, c_scale=0.1):
    out = []
    for p in list(main) + list(conj):
        out.append(_cx(g, L, 10.0 ** (-(p - 1) / 4.0)))
    out.append(_cx(g, 1, c_scale))
    return np.concatenate(out)


def _rel(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    den = max(np.linalg.norm(b), 1e-300)
    return np.linalg.norm(a - b) / den


CASES = [
    # (main orders, conj orders, L, n)
    ([1], [], 1, 1),
    ([1, 3, 5], [1, 3], 5, 37),        # Table 2 configuration
    ([1, 3, 5, 7], [1, 3, 5, 7], 4, 4),
    ([1, 3, 5, 7], [1, 3, 5, 7], 4, 3),
    ([1, 3, 5, 7], [1, 3, 5, 7], 4, 5),
    ([1, 5], [3], 3, 2),
    ([3, 7], [], 2, 19),
    ([1, 3, 5, 7, 9], [1, 3, 5, 7, 9], 8, 29),
]


# ---------------------------------------------------------------- forward ---

def pin_bruteforce_eq2(orc):
    """Oracle == first N rows of Psi @ h with Psi built as in Eq. (2)."""
    for i, (mo, co, L, n) in enumerate(CASES):
        g = _rng(100 + i)
        x = _cx(g, n, 0.6)
        h = _coeffs(g, mo, co, L)
        z = orc.forward(x, mo, co, L, h)
        zb = brute.forward_matrix(x, mo, co, L, h)
        assert _rel(z, zb) < 1e-13, (mo, co, L, n, _rel(z, zb))


def pin_bruteforce_history(orc):
    """With a carried history the oracle equals Eq. (2) applied to history ++ x."""
    for i, (mo, co, L, n) in enumerate(CASES):
        if L == 1:
            continue
        g = _rng(200 + i)
        x = _cx(g, n, 0.6)
        hist = _cx(g, L - 1, 0.6)
        h = _coeffs(g, mo, co, L)
        z = orc.forward(x, mo, co, L, h, hist=hist)
        zb = brute.forward_matrix(x, mo, co, L, h, hist=hist)
        assert _rel(z, zb) < 1e-13, (mo, co, L, n)


def pin_identity(orc):
    """h_{1,0} = 1, everything else 0: the predistorter is the identity, exactly."""
    g = _rng(1)
    x = _cx(g, 64, 0.5)
    mo, co, L = [1, 3, 5, 7], [1, 3, 5, 7], 4
    h = np.zeros((len(mo) + len(co)) * L + 1, dtype=np.complex128)
    h[0] = 1.0
    z = orc.forward(x, mo, co, L, h)
    assert np.array_equal(z, x)


def pin_single_coefficient(orc):
    """Only h_{p,k} = 1: z_n = psi_p(x_{n-k}) (and conj for a conjugate tap)."""
    g = _rng(2)
    n = 23
    x = _cx(g, n, 0.7)
    mo, co, L = [1, 3, 5], [1, 3], 4
    K = (len(mo) + len(co)) * L + 1
    for b, p in enumerate(mo + co):
        for k in range(L):
            h = np.zeros(K, dtype=np.complex128)
            h[b * L + k] = 1.0
            z = orc.forward(x, mo, co, L, h)
            ref = np.zeros(n, dtype=np.complex128)
            ref[k:] = brute.basis(x[:n - k], p)
            if b >= len(mo):
                ref = np.conj(ref)
            assert _rel(z, ref) < 1e-14, (p, k)
    h = np.zeros(K, dtype=np.complex128)
    h[-1] = 0.25 - 0.5j
    assert np.array_equal(orc.forward(x, mo, co, L, h), np.full(n, 0.25 - 0.5j))


def pin_linearity(orc):
    """Eq. (1) is linear in the coefficient vector."""
    g = _rng(3)
    mo, co, L = [1, 3, 5, 7], [1, 3, 5], 3
    x = _cx(g, 50, 0.5)
    h1 = _coeffs(g, mo, co, L)
    h2 = _coeffs(g, mo, co, L)
    a, b = 0.3 - 1.1j, -2.0 + 0.5j
    z = orc.forward(x, mo, co, L, a * h1 + b * h2)
    zl = a * orc.forward(x, mo, co, L, h1) + b * orc.forward(x, mo, co, L, h2)
    assert _rel(z, zl) < 1e-13


def pin_phase_equivariance(orc):
    """Without conjugate branches and c: D(e^{j t} x) = e^{j t} D(x); the conjugate
    branch alone gives D(e^{j t} x) = e^{-j t} D(x)."""
    g = _rng(4)
    x = _cx(g, 40, 0.5)
    rot = np.exp(1j * 0.7)
    mo, L = [1, 3, 5, 7], 5
    h = _coeffs(g, mo, [], L)
    h[-1] = 0.0
    z0 = orc.forward(x, mo, [], L, h)
    z1 = orc.forward(rot * x, mo, [], L, h)
    assert _rel(z1, rot * z0) < 1e-13
    co = [1, 3, 5]
    hc = _coeffs(g, [1], co, L)
    hc[:L] = 0.0
    hc[-1] = 0.0
    z0 = orc.forward(x, [1], co, L, hc)
    z1 = orc.forward(rot * x, [1], co, L, hc)
    assert _rel(z1, np.conj(rot) * z0) < 1e-13
    # and the mixed map is *not* equivariant (the conjugate branch matters)
    hm = _coeffs(g, mo, co, L)
    zm0 = orc.forward(x, mo, co, L, hm)
    zm1 = orc.forward(rot * x, mo, co, L, hm)
    assert _rel(zm1, rot * zm0) > 1e-3


def pin_conjugation_symmetry(orc):
    """With I_P = I_Q: conj(D_{h, hbar, c}(x)) = D_{conj hbar, conj h, conj c}(x)."""
    g = _rng(5)
    orders, L = [1, 3, 5], 4
    x = _cx(g, 33, 0.6)
    h = _coeffs(g, orders, orders, L)
    nb = len(orders) * L
    swapped = np.concatenate([np.conj(h[nb:2 * nb]), np.conj(h[:nb]), np.conj(h[-1:])])
    z = orc.forward(x, orders, orders, L, h)
    zs = orc.forward(x, orders, orders, L, swapped)
    assert _rel(np.conj(z), zs) < 1e-14


def pin_single_tone(orc):
    """x_n = A e^{j w n}: once the filters are full (n >= L-1),
    z_n = sum_p A^{p-1} H_p(e^{jw}) x_n + sum_q A^{q-1} G_q(e^{-jw}) conj(x_n) + c,
    with H_p, G_q the DTFTs of the tap vectors."""
    g = _rng(6)
    mo, co, L = [1, 3, 5, 7], [1, 3, 5], 6
    A, w, n = 0.8, 0.37, 64
    x = A * np.exp(1j * w * np.arange(n))
    h = _coeffs(g, mo, co, L)
    z = orc.forward(x, mo, co, L, h)
    k = np.arange(L)
    ref = np.full(n, h[-1], dtype=np.complex128)
    for b, p in enumerate(mo):
        Hp = np.sum(h[b * L:(b + 1) * L] * np.exp(-1j * w * k))
        ref = ref + A ** (p - 1) * Hp * x
    for b, q in enumerate(co):
        off = (len(mo) + b) * L
        Gq = np.sum(h[off:off + L] * np.exp(1j * w * k))
        ref = ref + A ** (q - 1) * Gq * np.conj(x)
    assert _rel(z[L - 1:], ref[L - 1:]) < 1e-13


def pin_constant_input(orc):
    """x_n = a for n >= 0: z_n uses the partial tap sums over k <= n."""
    g = _rng(7)
    mo, co, L = [1, 3, 5], [1, 3], 5
    a = 0.3 - 0.45j
    n = 12
    x = np.full(n, a)
    h = _coeffs(g, mo, co, L)
    z = orc.forward(x, mo, co, L, h)
    for t in range(n):
        kk = min(t, L - 1) + 1
        ref = h[-1]
        for b, p in enumerate(mo):
            ref += np.sum(h[b * L:b * L + kk]) * abs(a) ** (p - 1) * a
        for b, q in enumerate(co):
            off = (len(mo) + b) * L
            ref += np.sum(h[off:off + kk]) * abs(a) ** (q - 1) * np.conj(a)
        assert abs(z[t] - ref) <= 1e-14 * max(1.0, abs(ref)), t


def load_eq3_alpha():
    rows = []
    with open(os.path.join(GOLDEN, "eq3_warp_pa.txt")) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            p, re, im = line.split()
            rows.append((int(p), float(re) + 1j * float(im)))
    return rows


def pin_eq3_warp_pa(orc):
    """L = 1, I_P = {1,3,5}, h = alpha of Eq. (3), no conjugate branch, c = 0: the
    predistorter *is* the WARP PA model; evaluate it with numpy's polyval in |x|^2."""
    rows = load_eq3_alpha()
    orders = [p for p, _ in rows]
    alpha = np.array([a for _, a in rows])
    g = _rng(8)
    x = _cx(g, 200, 0.5)
    h = np.concatenate([alpha, [0.0]])
    z = orc.forward(x, orders, [], 1, h)
    ref = np.polynomial.polynomial.polyval(np.abs(x) ** 2, alpha) * x
    assert _rel(z, ref) < 1e-14


def pin_time_shift(orc):
    """Delaying the input by d samples (zero fill) delays the output; the first d
    outputs see only zeros and equal c."""
    g = _rng(9)
    mo, co, L = [1, 3, 5], [1, 3], 4
    x = _cx(g, 40, 0.5)
    h = _coeffs(g, mo, co, L)
    d = 7
    xs = np.concatenate([np.zeros(d), x])
    z = orc.forward(x, mo, co, L, h)
    zs = orc.forward(xs, mo, co, L, h)
    assert np.allclose(zs[:d], h[-1], rtol=0, atol=0)
    assert _rel(zs[d:], z) < 1e-14


def pin_chunked_history(orc):
    """Splitting a stream and carrying the last L-1 inputs gives the whole result."""
    g = _rng(10)
    mo, co, L = [1, 3, 5, 7], [1, 3, 5, 7], 6
    x = _cx(g, 101, 0.5)
    h = _coeffs(g, mo, co, L)
    z = orc.forward(x, mo, co, L, h)
    parts = []
    hist = np.zeros(L - 1, dtype=np.complex128)
    for a, b in [(0, 3), (3, 40), (40, 41), (41, 101)]:
        parts.append(orc.forward(x[a:b], mo, co, L, h, hist=hist))
        hist = np.concatenate([hist, x[a:b]])[-(L - 1):]
    assert _rel(np.concatenate(parts), z) < 1e-15


# --------------------------------------------------------------- backward ---

def _loss(orc, x, mo, co, L, h, W):
    """E = Re sum conj(W) z, so dE/dRe z + j dE/dIm z = W."""
    z = orc.forward(x, mo, co, L, h)
    return float(np.real(np.vdot(W, z)))


def pin_backward_fd(orc):
    """Central finite differences of E on Re and Im of every coefficient and of
    sampled inputs agree with the oracle gradient."""
    for i, (mo, co, L, n) in enumerate([([1, 3, 5], [1, 3], 3, 17), ([1, 3, 5, 7], [1, 3, 5, 7], 4, 11)]):
        g = _rng(300 + i)
        x = _cx(g, n, 0.7)
        h = _coeffs(g, mo, co, L)
        W = _cx(g, n)
        gx, gc = orc.backward(x, mo, co, L, h, W)
        eps = 1e-6
        fd = np.zeros_like(gc)
        for j in range(h.size):
            for unit, part in ((1.0, 0), (1j, 1)):
                hp = h.copy()
                hm = h.copy()
                hp[j] += unit * eps
                hm[j] -= unit * eps
                d = (_loss(orc, x, mo, co, L, hp, W) - _loss(orc, x, mo, co, L, hm, W)) / (2 * eps)
                fd[j] += d * (1.0 if part == 0 else 1j)
        assert _rel(gc, fd) < 1e-7, _rel(gc, fd)
        fdx = np.zeros_like(gx)
        for m in range(n):
            for unit, part in ((1.0, 0), (1j, 1)):
                xp = x.copy()
                xm = x.copy()
                xp[m] += unit * eps
                xm[m] -= unit * eps
                d = (_loss(orc, xp, mo, co, L, h, W) - _loss(orc, xm, mo, co, L, h, W)) / (2 * eps)
                fdx[m] += d * (1.0 if part == 0 else 1j)
        assert _rel(gx, fdx) < 1e-7, _rel(gx, fdx)


def pin_backward_dot(orc):
    """Eq. (1) is linear in the coefficients, so for any direction dh:
    Re <G, D_dh(x)> = Re <grad_h, dh>  (adjoint / dot-product test)."""
    g = _rng(11)
    mo, co, L = [1, 3, 5, 7], [1, 3, 5], 5
    x = _cx(g, 300, 0.5)
    h = _coeffs(g, mo, co, L)
    G = _cx(g, 300)
    _, gc = orc.backward(x, mo, co, L, h, G, want_dx=False)
    for _ in range(3):
        dh = _cx(g, h.size)
        lhs = np.real(np.vdot(G, orc.forward(x, mo, co, L, dh)))
        rhs = np.real(np.vdot(gc, dh))
        assert abs(lhs - rhs) <= 1e-12 * max(1.0, abs(lhs))


def pin_backward_autograd(orc):
    """Gradient of E through a plain PyTorch (float64, CPU) statement of Eq. (1)
    by torch.autograd equals the oracle's hand-derived adjoint."""
    import torch

    g = _rng(12)
    mo, co, L = [1, 3, 5], [1, 3], 4
    n = 57
    x = _cx(g, n, 0.6)
    h = _coeffs(g, mo, co, L)
    W = _cx(g, n)
    hist = _cx(g, L - 1, 0.6)
    gx, gc = orc.backward(x, mo, co, L, h, W, hist=hist)

    xt = torch.tensor(x, dtype=torch.complex128, requires_grad=True)
    ht = torch.tensor(h, dtype=torch.complex128, requires_grad=True)
    full = torch.cat([torch.tensor(hist, dtype=torch.complex128), xt])
    s = full.real ** 2 + full.imag ** 2
    z = torch.zeros(n, dtype=torch.complex128) + ht[-1]
    for b, p in enumerate(list(mo) + list(co)):
        basis = s ** ((p - 1) // 2) * full
        if b >= len(mo):
            basis = torch.conj(basis)
        for k in range(L):
            z = z + ht[b * L + k] * basis[L - 1 - k:L - 1 - k + n]
    E = torch.sum((torch.conj(torch.tensor(W)) * z).real)
    E.backward()
    assert _rel(gc, ht.grad.numpy()) < 1e-12
    assert _rel(gx, xt.grad.numpy()) < 1e-12


# ----------------------------------------------------- least squares (LS) ---

def pin_ls_normal(orc):
    """The normal equations equal Psi^H Psi and Psi^H t with Psi of Eq. (2) (first
    M rows), and solving them recovers coefficients that generated t exactly."""
    g = _rng(13)
    mo, co, L = [1, 3, 5], [1, 3], 3
    M = 80
    y = _cx(g, M, 0.6)
    h = _coeffs(g, mo, co, L)
    t = brute.forward_matrix(y, mo, co, L, h)
    A, b = orc.ls_normal(y, mo, co, L, t)
    P = brute.psi_matrix(y, mo, co, L)[:M]
    assert _rel(A, P.conj().T @ P) < 1e-13
    assert _rel(b, P.conj().T @ t) < 1e-13
    hh = np.linalg.solve(A, b)
    assert _rel(hh, h) < 1e-8


def pin_forward_at_matches_forward(orc):
    """Evaluating Eq. (1) at listed output indices gives exactly the entries of
    the whole-stream result at those indices (any order, repeats, the first and
    the last output), with and without a carried history."""
    g = _rng(14)
    mo, co, L = [1, 3, 5, 7], [1, 3, 5], 5
    n = 257
    x = _cx(g, n, 0.6)
    h = _coeffs(g, mo, co, L)
    idx = np.concatenate([[n - 1, 0, 1, 3, 3], g.integers(0, n, 40)])
    for hist in (None, _cx(g, L - 1, 0.6)):
        z = orc.forward(x, mo, co, L, h, hist=hist)
        za = orc.forward_at(x, mo, co, L, h, idx, hist=hist)
        assert np.array_equal(za, z[idx])


# ------------------------------------ transmitter chain (oracle/pa.py) ---
# The learning workload's loss: predistorter -> I/Q imbalance + LO leakage ->
# memory PA (Eq. 3 coefficients) -> E = mean |y/10 - x|^2.  The chain pins take
# the module holding ``chain_loss_and_gradient`` so the mutation tests can hand
# them planted copies of it.

CHAIN_ORDERS = ([1, 3, 5], [1, 3])
CHAIN_L = 3


def _pa_module(pa_mod):
    if pa_mod is None:
        import oracle.pa as pa_mod
    return pa_mod


def _chain_inputs(seed):
    """Two rows of 300 complex64 samples and coefficients away from any optimum."""
    g = _rng(seed)
    x = np.stack([_cx(g, 300, 0.3) for _ in range(2)]).astype(np.complex64)
    h = _coeffs(g, *CHAIN_ORDERS, CHAIN_L)
    h[0] += 1.0                       # near the identity, so the PA sees a sensible drive
    return x, h


def pin_chain_gradient_fd(orc, pa_mod=None):
    """dE/dcoeffs of the chain equals FP64 central differences of E on Re and Im
    of every coefficient (both rows summed)."""
    pa = _pa_module(pa_mod)
    x, h = _chain_inputs(400)
    E, gc = pa.chain_loss_and_gradient(orc, x, CHAIN_ORDERS, CHAIN_L, h)
    eps = 1e-6
    fd = np.zeros(h.size, dtype=np.complex128)
    for j in range(h.size):
        for unit in (1.0, 1j):
            hp = h.copy()
            hm = h.copy()
            hp[j] += unit * eps
            hm[j] -= unit * eps
            ep = pa.chain_loss_and_gradient(orc, x, CHAIN_ORDERS, CHAIN_L, hp)[0]
            em = pa.chain_loss_and_gradient(orc, x, CHAIN_ORDERS, CHAIN_L, hm)[0]
            fd[j] += (ep - em) / (2 * eps) * unit
    assert _rel(gc, fd) < 1e-7, _rel(gc, fd)


def pin_chain_loss_independent(orc, pa_mod=None):
    """The chain loss equals E rebuilt from the definitions by another route: the
    predistorter as Psi @ h of Eq. (2); the modulator as u = mu z + nu conj(z) +
    c_LO with mu = (1 + g e^{-j phi})/2, nu = (1 - g e^{j phi})/2 (g = 1.05,
    phi = 3 degrees, c_LO = 0.01 e^{j pi/4}); the PA as
    10 sum_p alpha_p (beta * psi_p(u)) with the Eq. (3) coefficients of the
    golden file and the memory taps beta = [1, -0.08+0.04j, 0.02-0.01j], by
    numpy convolution.  Stage coefficients are rounded to complex64, as the
    library receives them."""
    pa = _pa_module(pa_mod)
    x, h = _chain_inputs(401)
    E, _ = pa.chain_loss_and_gradient(orc, x, CHAIN_ORDERS, CHAIN_L, h)
    alpha = dict(load_eq3_alpha())
    beta = np.array([1.0, -0.08 + 0.04j, 0.02 - 0.01j])
    amp, phi = 1.05, np.deg2rad(3.0)
    mu = complex(np.complex64((1 + amp * np.exp(-1j * phi)) / 2))
    nu = complex(np.complex64((1 - amp * np.exp(1j * phi)) / 2))
    lo = complex(np.complex64(0.01 * np.exp(1j * np.pi / 4)))
    total = 0.0
    for row in x:
        z = brute.forward_matrix(row, *CHAIN_ORDERS, CHAIN_L, h)
        u = mu * z + nu * np.conj(z) + lo
        y = np.zeros_like(u)
        for p in (1, 3, 5):
            taps = (10.0 * alpha[p] * beta).astype(np.complex64).astype(np.complex128)
            y += np.convolve(brute.basis(u, p), taps)[:u.size]
        total += float(np.sum(np.abs(y / 10.0 - row.astype(np.complex128)) ** 2))
    ref = total / x.size
    assert abs(E - ref) <= 1e-11 * ref, (E, ref)


# ------------------------------ indirect learning (oracle/ila.py) ---------

def _ila_module(ila_mod):
    if ila_mod is None:
        import oracle.ila as ila_mod
    return ila_mod


def pin_ila_inverts_widely_linear_transmitter(orc, ila_mod=None):
    """A transmitter u = mu z + nu conj(z) + c_LO followed by a complex gain G a
    has an exact inverse in the basis (order 1 in both branches, c):
    h_1 = conj(mu) / (a D), hbar_1 = -nu / (conj(a) D),
    c = -(conj(mu) c_LO - nu conj(c_LO)) / D with D = |mu|^2 - |nu|^2, every
    other coefficient 0.  One iteration from the identity must find it, and the
    linearization error must then vanish."""
    ila = _ila_module(ila_mod)
    g = _rng(15)
    mu, nu, lo = 0.97 + 0.05j, 0.03 - 0.02j, 0.02 - 0.01j
    G, a = 10.0, 0.8 * np.exp(0.3j)
    stages = [([1], [1], 1, np.array([mu, nu, lo])), ([1], [], 1, np.array([G * a, 0.0]))]
    orders, L = ([1, 3, 5], [1, 3]), 2
    x = np.stack([_cx(g, 400, 0.4) for _ in range(2)])
    K = (len(orders[0]) + len(orders[1])) * L + 1
    h0 = np.zeros(K, dtype=np.complex128)
    h0[0] = 1.0
    D = abs(mu) ** 2 - abs(nu) ** 2
    ref = np.zeros(K, dtype=np.complex128)
    ref[0] = np.conj(mu) / (a * D)
    ref[len(orders[0]) * L] = -nu / (np.conj(a) * D)
    ref[-1] = -(np.conj(mu) * lo - nu * np.conj(lo)) / D
    errs, hs = ila.run(orc, x, orders, L, h0, 1, ridge=0.0, gain=G, stages=stages)
    assert _rel(hs[0], ref) < 1e-9, _rel(hs[0], ref)
    assert errs[1] < -200.0, errs


def pin_ila_least_squares_route(orc, ila_mod=None):
    """From coefficients away from the identity, one iteration on the synthetic
    transmitter equals the ridge least-squares fit by another route: numpy's
    lstsq of [Psi; sqrt(delta) I] h = [z; 0], with Psi the Eq. (2) basis matrix
    of PA output / 10 (first M rows per row of input, stacked) and z the
    predistorter output, delta = ridge * mean(Re diag Psi^H Psi)."""
    import oracle.pa as opa

    ila = _ila_module(ila_mod)
    g = _rng(16)
    orders, L = ([1, 3, 5], [1, 3]), 3
    x = np.stack([_cx(g, 300, 0.25) for _ in range(2)]).astype(np.complex64)
    h = 0.02 * _coeffs(g, *orders, L)
    h[0] += 1.0
    ridge = 1e-3
    Ps, zs = [], []
    for row in x:
        z = brute.forward_matrix(row, *orders, L, h)
        y = z
        for smo, sco, sL, sh in opa.stages():
            y = orc.forward(y, smo, sco, sL, sh)
        Ps.append(brute.psi_matrix(y / 10.0, *orders, L)[:row.size])
        zs.append(z)
    P = np.concatenate(Ps)
    t = np.concatenate(zs)
    delta = ridge * float(np.mean(np.real(np.diag(P.conj().T @ P))))
    K = P.shape[1]
    Pa = np.concatenate([P, np.sqrt(delta) * np.eye(K)])
    ta = np.concatenate([t, np.zeros(K)])
    ref = np.linalg.lstsq(Pa, ta, rcond=None)[0]
    hn = ila.iteration(orc, x, orders, L, h, ridge=ridge)
    assert _rel(hn, ref) < 1e-8, _rel(hn, ref)


ALL_PINS = [v for k, v in sorted(globals().items()) if k.startswith("pin_")]
CHAIN_PINS = [pin_chain_gradient_fd, pin_chain_loss_independent]
ILA_PINS = [pin_ila_inverts_widely_linear_transmitter, pin_ila_least_squares_route]
