"""FP64 reference of the learned Metropolis proposal (a 3-layer tanh MLP).

TEST INFRASTRUCTURE ONLY.

Network: x (3N raw electron coordinates) -> h1 = tanh(x W1 + b1) -> h2 =
tanh(h1 W2 + b2) -> o = h2 W3 + b3 (4N outputs): mu = o[:3N] (per-electron
move mean), ls = clip(o[3N:], ln 0.01, ln 2) (per-electron log step),
sigma = exp(ls).  Parameters are one flat vector laid out as
[W1 (in x h), b1 (h), W2 (h x h), b2 (h), W3 (h x out), b3 (out)], row-major.

Proposal: R' = R + mu(R) + sigma(R) xi, xi ~ N(0, I).  Exact Metropolis-
Hastings acceptance A = min(1, exp(l)) with
   l = 2 (ln|Psi(R')| - ln|Psi(R)|) + ln q(R|R') - ln q(R'|R),
   ln q(B|A) = sum_e [ -|B_e - A_e - mu_e(A)|^2 / (2 sigma_e(A)^2) - 3 ls_e(A) ].
Training objective (expected squared jump distance with the exact
acceptance): J = mean_w A_w |R'_w - R_w|^2, maximised; loss = -J.
"""
from __future__ import annotations

import numpy as np

LS_MIN, LS_MAX = float(np.log(0.01)), float(np.log(2.0))


def shapes(n_in, n_hid, n_out):
    return [(n_in, n_hid), (n_hid,), (n_hid, n_hid), (n_hid,), (n_hid, n_out), (n_out,)]


def n_params(n_in, n_hid, n_out):
    return sum(int(np.prod(s)) for s in shapes(n_in, n_hid, n_out))


def unpack(flat, n_in, n_hid, n_out):
    out, o = [], 0
    for s in shapes(n_in, n_hid, n_out):
        k = int(np.prod(s))
        out.append(np.asarray(flat[o:o + k], dtype=np.float64).reshape(s))
        o += k
    return out


def pack(parts):
    return np.concatenate([np.asarray(p, dtype=np.float64).ravel() for p in parts])


def forward(flat, X, n_hid, n_out):
    n_in = X.shape[1]
    W1, b1, W2, b2, W3, b3 = unpack(flat, n_in, n_hid, n_out)
    h1 = np.tanh(X @ W1 + b1)
    h2 = np.tanh(h1 @ W2 + b2)
    o = h2 @ W3 + b3
    return o, (X, h1, h2)


def backward(flat, cache, dO, n_hid, n_out):
    """Parameter gradient (flat) and input gradient of sum(dO * o)."""
    X, h1, h2 = cache
    n_in = X.shape[1]
    W1, b1, W2, b2, W3, b3 = unpack(flat, n_in, n_hid, n_out)
    dW3 = h2.T @ dO
    db3 = dO.sum(0)
    dh2 = dO @ W3.T
    dz2 = dh2 * (1.0 - h2 * h2)
    dW2 = h1.T @ dz2
    db2 = dz2.sum(0)
    dh1 = dz2 @ W2.T
    dz1 = dh1 * (1.0 - h1 * h1)
    dW1 = X.T @ dz1
    db1 = dz1.sum(0)
    dX = dz1 @ W1.T
    return pack([dW1, db1, dW2, db2, dW3, db3]), dX


def head(o, N):
    mu = o[:, :3 * N].reshape(-1, N, 3)
    raw = o[:, 3 * N:]
    ls = np.clip(raw, LS_MIN, LS_MAX)
    inside = (raw > LS_MIN) & (raw < LS_MAX)
    return mu, ls, inside


def adam(flat, grad, m, v, t, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam step (bias-corrected), t = 1-based step count."""
    m = b1 * m + (1 - b1) * grad
    v = b2 * v + (1 - b2) * grad * grad
    mh = m / (1 - b1 ** t)
    vh = v / (1 - b2 ** t)
    return flat - lr * mh / (np.sqrt(vh) + eps), m, v


def log_q(Rb, Ra, mu_a, ls_a):
    """ln q(Rb | Ra) up to a constant, per walker."""
    d = Rb - Ra - mu_a
    return np.sum(-np.sum(d * d, axis=2) / (2.0 * np.exp(2.0 * ls_a)) - 3.0 * ls_a, axis=1)


def coulomb_potential(R, Z):
    """V = -Z sum_e 1/|r_e| + sum_{e<f} 1/|r_e - r_f| per walker and its
    gradient [B][N][3] (nucleus of charge Z at the origin)."""
    r = np.linalg.norm(R, axis=2)
    V = -Z * np.sum(1.0 / r, axis=1)
    g = Z * R / r[:, :, None] ** 3
    N = R.shape[1]
    for e in range(N):
        for f in range(e + 1, N):
            d = R[:, e] - R[:, f]
            dn = np.linalg.norm(d, axis=1)
            V += 1.0 / dn
            c = (d / dn[:, None] ** 3)
            g[:, e] -= c
            g[:, f] += c
    return V, g


def esjd_loss_and_grad(flat, R, xi, logpsi_R, psi_fn, n_hid, jump_ref=0.0, objective=0, Z=0.0):
    """Loss -mean(A jump) and its exact gradient w.r.t. the parameters:
    objective 0, jump = sum_e c_e |r'_e - r_e|^2 with c_e = 1, or
    1 / (|r_e|^2 + jump_ref^2) when jump_ref > 0; objective 1,
    jump = (V(R') - V(R))^2 with V the Coulomb potential (nuclear charge Z).

    R [B][N][3], xi [B][N][3]; logpsi_R [B] = ln|Psi(R)|; psi_fn(R') returns
    (ln|Psi(R')| [B], grad ln|Psi(R')| [B][N][3]).  Returns (loss, grad, info).
    """
    B, N, _ = R.shape
    n_out = 4 * N
    X = R.reshape(B, 3 * N)
    o, c1 = forward(flat, X, n_hid, n_out)
    mu, ls, in1 = head(o, N)
    sig = np.exp(ls)[:, :, None]
    Rp = R + mu + sig * xi
    lp, glp = psi_fn(Rp)
    o2, c2 = forward(flat, Rp.reshape(B, 3 * N), n_hid, n_out)
    mu2, ls2, in2 = head(o2, N)
    lq_fwd = np.sum(-0.5 * np.sum(xi * xi, axis=2) - 3.0 * ls, axis=1)   # ln q(R'|R)
    d = R - Rp - mu2
    s2 = np.exp(2.0 * ls2)[:, :, None]
    lq_rev = np.sum(-np.sum(d * d, axis=2) / (2.0 * np.exp(2.0 * ls2)) - 3.0 * ls2, axis=1)
    ell = 2.0 * (lp - logpsi_R) + lq_rev - lq_fwd
    A = np.minimum(1.0, np.exp(np.minimum(ell, 0.0)))
    if objective == 1:
        Vp, dVp = coulomb_potential(Rp, Z)
        dv = Vp - coulomb_potential(R, Z)[0]
        jump = dv * dv
        djump = 2.0 * dv[:, None, None] * dVp
    else:
        cw = np.ones((B, N)) if jump_ref <= 0 else 1.0 / (np.sum(R * R, axis=2) + jump_ref ** 2)
        jump = np.sum(cw * np.sum((Rp - R) ** 2, axis=2), axis=1)
        djump = 2.0 * cw[:, :, None] * (Rp - R)
    J = A * jump
    loss = -np.mean(J)
    # d loss / d J_w = -1/B
    gJ = -np.ones(B) / B
    g_ell = gJ * np.where(ell < 0.0, A, 0.0) * jump
    g_Rp = gJ[:, None, None] * A[:, None, None] * djump
    # ell: 2 lnPsi(R') + lq_rev(R', mu2, ls2) - lq_fwd(ls)
    g_Rp += g_ell[:, None, None] * (2.0 * glp + d / s2)
    g_mu2 = g_ell[:, None, None] * (d / s2)
    g_ls2 = g_ell[:, None] * (np.sum(d * d, axis=2) / np.exp(2.0 * ls2) - 3.0) * in2
    dO2 = np.concatenate([g_mu2.reshape(B, 3 * N), g_ls2], axis=1)
    gp2, gX2 = backward(flat, c2, dO2, n_hid, n_out)
    g_Rp += gX2.reshape(B, N, 3)
    # R' = R + mu + sigma xi
    g_mu = g_Rp
    g_ls = (np.sum(g_Rp * sig * xi, axis=2) + g_ell[:, None] * 3.0) * in1
    dO1 = np.concatenate([g_mu.reshape(B, 3 * N), g_ls], axis=1)
    gp1, _ = backward(flat, c1, dO1, n_hid, n_out)
    info = dict(A=A, ell=ell, Rp=Rp, jump=jump)
    return loss, gp1 + gp2, info
