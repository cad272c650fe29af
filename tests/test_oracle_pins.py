"""Pins of the FP64 oracle against closed forms, brute force, textbook
identities and high-precision arithmetic.  None of these recomputes the
oracle's own formulas: each reaches the same quantity by another route."""
import itertools
import math

import numpy as np
import pytest

import oracle
from oracle import brute
from gen.workloads import Workload, encode, make_config, make_custom


def _one_orbital_wl(pw, alpha, coef):
    pw = np.array(pw, dtype=np.int32).reshape(1, -1, 3)
    a = np.array(alpha, dtype=np.float64).reshape(1, -1)
    c = np.array(coef, dtype=np.float64).reshape(1, -1)
    return Workload("one", 1, 0, 1, pw.shape[1], pw, a, c, 1,
                    np.zeros((1, 1), np.uint64), np.zeros((1, 1), np.uint64),
                    np.ones(1), np.zeros((1, 1, 3)))


# ---------------------------------------------------------------- orbitals

@pytest.mark.parametrize("r", [(0.3, -0.7, 1.1), (0.0, 0.0, 0.0), (2.0, 0.0, -1.5)])
def test_orbital_closed_forms(r):
    x, y, z = r
    r2 = x * x + y * y + z * z
    al = 0.8
    g = math.exp(-al * r2)
    # s: phi = g ; grad = -2 al r g ; lap = (4 al^2 r^2 - 6 al) g
    o = oracle.orbitals(_one_orbital_wl([0, 0, 0], [al], [1.0]), r)[:, 0]
    np.testing.assert_allclose(o, [g, -2 * al * x * g, -2 * al * y * g, -2 * al * z * g,
                                   (4 * al * al * r2 - 6 * al) * g], rtol=1e-14, atol=1e-300)
    # p_x: phi = x g ; d/dx = (1 - 2 al x^2) g ; lap = x g (4 al^2 r^2 - 10 al)
    o = oracle.orbitals(_one_orbital_wl([1, 0, 0], [al], [1.0]), r)[:, 0]
    np.testing.assert_allclose(o, [x * g, (1 - 2 * al * x * x) * g, -2 * al * x * y * g,
                                   -2 * al * x * z * g, x * g * (4 * al * al * r2 - 10 * al)],
                               rtol=1e-13, atol=1e-15)
    # d_xx: phi = x^2 g ; lap = g (2 - 14 al x^2 + 4 al^2 r^2 x^2) (product rule)
    o = oracle.orbitals(_one_orbital_wl([2, 0, 0], [al], [1.0]), r)[:, 0]
    np.testing.assert_allclose(o[[0, 1, 4]],
                               [x * x * g, (2 * x - 2 * al * x ** 3) * g,
                                g * (2 - 14 * al * x * x + 4 * al * al * r2 * x * x)],
                               rtol=1e-13, atol=1e-15)
    # d_xy: phi = x y g ; lap = x y g (4 al^2 r^2 - 14 al)
    o = oracle.orbitals(_one_orbital_wl([1, 1, 0], [al], [1.0]), r)[:, 0]
    np.testing.assert_allclose(o[[0, 4]], [x * y * g, x * y * g * (4 * al * al * r2 - 14 * al)],
                               rtol=1e-13, atol=1e-15)


def test_orbital_derivatives_finite_differences():
    wl = make_config(2)
    rng = np.random.default_rng(3)
    for _ in range(4):
        r = rng.normal(0, 1.0, 3)
        o = oracle.orbitals(wl, r)
        h = 1e-3

        def val(rr):
            return oracle.orbitals(wl, rr)[0]

        lap = np.zeros(wl.n_mo)
        for ax in range(3):
            def d1(hh):
                e = np.zeros(3); e[ax] = hh
                return (val(r + e) - val(r - e)) / (2 * hh)

            def d2(hh):
                e = np.zeros(3); e[ax] = hh
                return (val(r + e) - 2 * val(r) + val(r - e)) / (hh * hh)
            g_fd = (4 * d1(h / 2) - d1(h)) / 3          # Richardson
            np.testing.assert_allclose(o[1 + ax], g_fd, rtol=1e-6, atol=1e-8)
            lap += (4 * d2(h / 2) - d2(h)) / 3
        np.testing.assert_allclose(o[4], lap, rtol=1e-4, atol=1e-5)


# ---------------------------------------------------------- one determinant

@pytest.mark.parametrize("n", [1, 2, 3, 4, 5])
def test_slater_vs_leibniz(n):
    rng = np.random.default_rng(n)
    for trial in range(5):
        S = rng.normal(size=(n, n))
        S *= 2.0 ** rng.integers(-300, 300, size=n)    # wildly scaled columns
        G = rng.normal(size=(4, n, n)) * (S[None] != 0)
        G = G * (np.abs(S).max(axis=0))[None, None, :]
        sg, la, rt = oracle.slater(S, G)
        D, g = brute.det_and_grad((S / np.abs(S).max(axis=0)).tolist(),
                                  (G / np.abs(S).max(axis=0)).tolist())
        scale = np.sum(np.log(np.abs(S).max(axis=0)))
        assert sg == np.sign(D)
        assert abs(la - (math.log(abs(D)) + scale)) < 1e-12 * max(1.0, abs(la))
        # row-replacement identity: grad~_e D / D
        np.testing.assert_allclose(rt, g / D, rtol=1e-11, atol=1e-11 * np.abs(g / D).max())


def test_slater_vs_slogdet_and_singular():
    rng = np.random.default_rng(9)
    S = rng.normal(size=(9, 9))
    sg, la, _ = oracle.slater(S, np.zeros((4, 9, 9)))
    s2, l2 = np.linalg.slogdet(S)
    assert sg == s2 and abs(la - l2) < 1e-13
    S[3] = S[5]                                     # two equal rows -> exactly singular
    S[3, :] = S[5, :]
    sg, la, rt = oracle.slater(np.array(S), np.ones((4, 9, 9)))
    assert sg == 0.0 or abs(la - np.linalg.slogdet(S)[1]) < 1e-6


def test_sherman_morrison_column_update():
    # Eq. (sherman): replacing column k by u gives det ratio 1 + v_k^T S^-1 (u - S e_k)
    rng = np.random.default_rng(4)
    n = 7
    S = rng.normal(size=(n, n))
    Sinv = np.linalg.inv(S)
    for k in range(n):
        newcol = rng.normal(size=n)
        ratio_sm = 1.0 + Sinv[k] @ (newcol - S[:, k])
        S2 = S.copy(); S2[:, k] = newcol
        _, la1, _ = oracle.slater(S, np.zeros((4, n, n)))
        s2, la2, _ = oracle.slater(S2, np.zeros((4, n, n)))
        s1 = oracle.slater(S, np.zeros((4, n, n)))[0]
        assert abs(s1 * s2 * math.exp(la2 - la1) - ratio_sm) < 1e-12 * max(1, abs(ratio_sm))
        # the SM-updated inverse, (S + u v_k^T)^-1, inverts S2
        u = newcol - S[:, k]
        Sinv2 = Sinv - np.outer(Sinv @ u, Sinv[k]) / (1 + Sinv[k] @ u)
        np.testing.assert_allclose(Sinv2 @ S2, np.eye(n), atol=1e-10)


# ---------------------------------------------------------- whole wavefunction

def _scaled_errors(res, psi_s, logabs_s, gl_s, w):
    ep = abs(psi_s * res.sign[w] * math.exp(logabs_s - res.logabs[w]) - 1) / res.rs_psi[w]
    eg = np.max(np.abs(gl_s - res.gl[w]) / res.rs_gl[w])
    return ep, eg


def test_tiny_config_vs_leibniz_brute_force():
    wl = make_config(1)
    res = oracle.evaluate(wl, n_threads=2)
    for w in range(wl.n_walk):
        psi, grad = brute.psi_brute(wl, wl.R[w])
        ep, eg = _scaled_errors(res, np.sign(psi), math.log(abs(psi)), grad / psi, w)
        assert ep < 1e-12 and eg < 1e-12, (w, ep, eg)


def test_error_scales_vs_brute_force():
    """rs_psi = S_Psi / |Psi| and rs_gl = S_grad / |Psi|, with S the sums of
    the absolute values of the terms of Eq. (1) and of Eq. (nabla) (Sec. 2.3),
    recomputed product by product with Leibniz determinants.  These scales are
    the denominators of every parity gate, so they are pinned here."""
    wl = make_config(1)
    res = oracle.evaluate(wl, n_threads=2)
    for w in range(wl.n_walk):
        psi, _, s_psi, s_grad = brute.psi_brute(wl, wl.R[w], with_abs=True)
        assert abs(res.rs_psi[w] - s_psi / abs(psi)) <= 1e-12 * res.rs_psi[w], w
        np.testing.assert_allclose(res.rs_gl[w], s_grad / abs(psi), rtol=1e-12, atol=0)
        # a sum of absolute values bounds the absolute value of the sum
        assert res.rs_psi[w] >= 1.0 - 1e-14
        assert np.all(res.rs_gl[w] * abs(psi) >= np.abs(res.gl[w] * psi) * (1 - 1e-12))


def _cauchy_binet_case(n_mo, n_up, n_dn, n_walk, seed):
    base = make_custom(n_up, n_dn, n_mo, 3, 2, 2, (1,), 1, n_walk, sigma=1.0, seed=seed,
                       alpha_range=(0.2, 2.0))
    rng = np.random.default_rng(seed)
    Bu = rng.normal(size=(n_mo, n_up))
    Bd = rng.normal(size=(n_mo, n_dn))
    I_all = list(itertools.combinations(range(n_mo), n_up))
    J_all = list(itertools.combinations(range(n_mo), n_dn))
    du = np.array([np.linalg.det(Bu[list(I)]) for I in I_all])
    dd = np.array([np.linalg.det(Bd[list(J)]) for J in J_all])
    wu = encode(I_all, base.n_int)
    wd = encode(J_all, base.n_int)
    ii, jj = np.meshgrid(np.arange(len(I_all)), np.arange(len(J_all)), indexing="ij")
    ii, jj = ii.ravel(), jj.ravel()
    base.det_up = np.ascontiguousarray(wu[ii])
    base.det_dn = np.ascontiguousarray(wd[jj])
    base.c = du[ii] * dd[jj]
    return base, Bu, Bd


@pytest.mark.parametrize("shape", [(8, 4, 3, 3), (12, 6, 5, 2)])
def test_cauchy_binet_full_ci(shape):
    """sum_{I,J} detB_up[I] detB_dn[J] D_I D_J = det(Phi_up B_up) det(Phi_dn B_dn)."""
    n_mo, n_up, n_dn, W = shape
    wl, Bu, Bd = _cauchy_binet_case(n_mo, n_up, n_dn, W, seed=n_mo)
    res = oracle.evaluate(wl, n_threads=4)
    for w in range(W):
        orb = np.array([oracle.orbitals(wl, wl.R[w, e]) for e in range(wl.n_elec)])
        sgn, logabs = 1.0, 0.0
        gl = np.zeros((wl.n_elec, 4))
        for e0, n, B in ((0, n_up, Bu), (n_up, n_dn, Bd)):
            Pm = orb[e0:e0 + n, 0, :] @ B                     # n x n
            s, l = np.linalg.slogdet(Pm)
            sgn *= s
            logabs += l
            Pinv = np.linalg.inv(Pm)
            for q in range(4):
                Gq = orb[e0:e0 + n, 1 + q, :] @ B
                gl[e0:e0 + n, q] = np.einsum("ce,ec->e", Pinv, Gq)
        assert res.sign[w] == sgn
        assert abs(res.logabs[w] - logabs) < 1e-11 * (1 + res.rs_psi[w])
        np.testing.assert_allclose(res.gl[w], gl, rtol=0, atol=1e-10 * (1 + np.abs(gl).max()))


def test_error_scales_cauchy_binet_closed_form():
    """For c_IJ = det B_up[I] det B_dn[J] the absolute-term sums factorise:
    S_Psi = S_up S_dn with S_sigma = sum_I |det B_sigma[I]| |det Phi_sigma[:, I]|,
    and for an up electron S_grad[e,q] = (sum_I |det B_up[I]| |grad~_eq det
    Phi_up[:, I]|) S_dn, the derivative determinant taken by row replacement
    (numpy LU, independent of the oracle).  Checks rs_psi and rs_gl at the
    scale of hundreds of products."""
    n_mo, n_up, n_dn, W = 8, 4, 3, 3
    wl, Bu, Bd = _cauchy_binet_case(n_mo, n_up, n_dn, W, seed=n_mo)
    res = oracle.evaluate(wl, n_threads=4)
    for w in range(W):
        orb = np.array([oracle.orbitals(wl, wl.R[w, e]) for e in range(wl.n_elec)])
        S_spin, G_spin, psi = [], [], 1.0
        for e0, n, B in ((0, n_up, Bu), (n_up, n_dn, Bd)):
            subsets = list(itertools.combinations(range(n_mo), n))
            cB = np.array([abs(np.linalg.det(B[list(I)])) for I in subsets])
            mats = np.array([orb[e0:e0 + n, 0][:, list(I)] for I in subsets])   # [nI][n][n]
            D = np.linalg.det(mats)
            psi *= np.linalg.det(orb[e0:e0 + n, 0, :] @ B)
            S_spin.append(np.sum(cB * np.abs(D)))
            g = np.zeros((n, 4))
            for e in range(n):
                for q in range(4):
                    rep = mats.copy()
                    rep[:, e, :] = orb[e0 + e, 1 + q][np.array(subsets)]
                    g[e, q] = np.sum(cB * np.abs(np.linalg.det(rep)))
            G_spin.append(g)
        s_psi = S_spin[0] * S_spin[1]
        s_grad = np.concatenate([G_spin[0] * S_spin[1], G_spin[1] * S_spin[0]])
        assert abs(res.rs_psi[w] - s_psi / abs(psi)) <= 1e-10 * res.rs_psi[w], w
        np.testing.assert_allclose(res.rs_gl[w], s_grad / abs(psi), rtol=1e-10, atol=0)


def test_eq1_equals_bilinear_form():
    for cid in (1, 2, 3):
        wl = make_config(cid)
        R = wl.R[:6]
        a = oracle.evaluate(wl, R, mode=0, n_threads=4)
        b = oracle.evaluate(wl, R, mode=1, n_threads=4)
        assert np.array_equal(a.sign, b.sign)
        assert np.all(np.abs(a.logabs - b.logabs) < 1e-12 * a.rs_psi)
        assert np.all(np.abs(a.gl - b.gl) < 1e-11 * a.rs_gl)


def test_finite_differences_of_log_psi():
    wl = make_config(2)
    for w in range(3):
        R0 = wl.R[w].copy()
        base = oracle.evaluate(wl, R0[None], n_threads=2)
        h = 2e-3

        def logpsi(dR):
            r = oracle.evaluate(wl, (R0 + dR)[None], n_threads=1)
            return r.logabs[0]

        for e in range(0, wl.n_elec, 4):
            lap_log = 0.0
            grad = np.zeros(3)
            for ax in range(3):
                def d1(hh):
                    d = np.zeros_like(R0); d[e, ax] = hh
                    return (logpsi(d) - logpsi(-d)) / (2 * hh)

                def d2(hh):
                    d = np.zeros_like(R0); d[e, ax] = hh
                    return (logpsi(d) - 2 * base.logabs[0] + logpsi(-d)) / (hh * hh)
                grad[ax] = (4 * d1(h / 2) - d1(h)) / 3
                lap_log += (4 * d2(h / 2) - d2(h)) / 3
            g = base.gl[0, e, :3]
            np.testing.assert_allclose(g, grad, rtol=1e-6, atol=1e-6 * np.abs(g).max())
            lap = lap_log + grad @ grad                  # Psi''/Psi = (ln Psi)'' + (ln Psi)'^2
            assert abs(base.gl[0, e, 3] - lap) < 1e-4 * max(1.0, abs(lap))


def test_antisymmetry_same_spin_swap():
    wl = make_config(2)
    R = wl.R[:4].copy()
    a = oracle.evaluate(wl, R, n_threads=2)
    for (e1, e2) in ((0, 3), (wl.n_up, wl.n_up + 2)):
        R2 = R.copy()
        R2[:, [e1, e2]] = R2[:, [e2, e1]]
        b = oracle.evaluate(wl, R2, n_threads=2)
        assert np.array_equal(b.sign, -a.sign)
        np.testing.assert_allclose(b.logabs, a.logabs, rtol=0, atol=1e-12 * np.abs(a.logabs).max())
        perm = list(range(wl.n_elec)); perm[e1], perm[e2] = e2, e1
        np.testing.assert_allclose(b.gl, a.gl[:, perm], rtol=0, atol=1e-10 * a.rs_gl.max())


def test_spin_swap_symmetry():
    wl = make_custom(4, 4, 14, 3, 20, 20, (1, 2), 150, 3, seed=21)
    # symmetric C: use the same unique lists for both spins and add transposed products
    wl.det_dn = wl.det_up.copy()
    words = np.unique(wl.det_up, axis=0)
    rng = np.random.default_rng(2)
    pairs = set()
    while len(pairs) < 60:
        i, j = rng.integers(0, len(words), 2)
        pairs.add((min(i, j), max(i, j)))
    up, dn, c = [], [], []
    for (i, j) in sorted(pairs):
        v = rng.normal()
        up.append(words[i]); dn.append(words[j]); c.append(v)
        if i != j:
            up.append(words[j]); dn.append(words[i]); c.append(v)
    wl.det_up, wl.det_dn, wl.c = np.array(up), np.array(dn), np.array(c)
    a = oracle.evaluate(wl, n_threads=2)
    R2 = np.concatenate([wl.R[:, 4:], wl.R[:, :4]], axis=1)
    b = oracle.evaluate(wl, R2, n_threads=2)
    assert np.array_equal(a.sign, b.sign)
    np.testing.assert_allclose(a.logabs, b.logabs, rtol=1e-13)
    np.testing.assert_allclose(b.gl, np.concatenate([a.gl[:, 4:], a.gl[:, :4]], axis=1),
                               atol=1e-11 * a.rs_gl.max())


def test_linearity_in_coefficients():
    wl = make_config(2)
    R = wl.R[:4]
    rng = np.random.default_rng(8)
    c1 = wl.c.copy()
    c2 = rng.normal(size=wl.n_det) * 0.01
    a = oracle.evaluate(wl, R, c=c1, n_threads=2)
    b = oracle.evaluate(wl, R, c=c2, n_threads=2)
    s = oracle.evaluate(wl, R, c=c1 + c2, n_threads=2)
    lin = a.sign * np.exp(a.logabs - s.logabs) + b.sign * np.exp(b.logabs - s.logabs)
    np.testing.assert_allclose(lin, s.sign, rtol=0, atol=1e-11 * (1 + a.rs_psi.max() + b.rs_psi.max()))
    # derivatives add in the same way
    glin = (a.gl * (a.sign * np.exp(a.logabs - s.logabs))[:, None, None]
            + b.gl * (b.sign * np.exp(b.logabs - s.logabs))[:, None, None])
    np.testing.assert_allclose(glin, s.gl * s.sign[:, None, None], atol=1e-9 * np.abs(s.gl).max())


def test_single_product_is_textbook_slater():
    wl = make_config(2)
    k = 37
    R = wl.R[:5]
    r = oracle.evaluate(wl, R, c=np.array([0.3]), det_up=wl.det_up[k:k + 1],
                        det_dn=wl.det_dn[k:k + 1], n_threads=2)
    from oracle.preprocess import occupied
    ou, od = occupied(wl.det_up[k]), occupied(wl.det_dn[k])
    for w in range(5):
        orb = np.array([oracle.orbitals(wl, R[w, e]) for e in range(wl.n_elec)])
        tot_l, tot_s = math.log(0.3), 1.0
        for e0, n, o in ((0, wl.n_up, ou), (wl.n_up, wl.n_dn, od)):
            S = orb[e0:e0 + n, 0][:, o]
            s, l = np.linalg.slogdet(S)
            tot_l += l; tot_s *= s
            Sinv = np.linalg.inv(S)
            for q in range(4):
                gq = np.einsum("ce,ec->e", Sinv, orb[e0:e0 + n, 1 + q][:, o])
                np.testing.assert_allclose(r.gl[w, e0:e0 + n, q], gq, rtol=1e-9, atol=1e-9)
        assert r.sign[w] == tot_s and abs(r.logabs[w] - tot_l) < 1e-10


def test_high_precision_mpmath_tiny():
    """FP64 oracle within 1e-13 of a 40-digit evaluation of Eq. (1)."""
    mpmath = pytest.importorskip("mpmath")
    mpmath.mp.dps = 40
    wl = make_config(1)
    res = oracle.evaluate(wl, wl.R[:2], n_threads=1)
    from oracle.preprocess import occupied
    for w in range(2):
        orb = [oracle.orbitals(wl, wl.R[w, e]) for e in range(wl.n_elec)]
        cache = {}

        def D(words, e0, n):
            key = (tuple(int(x) for x in words), e0)
            if key not in cache:
                o = occupied(words)
                M = mpmath.matrix([[mpmath.mpf(orb[e0 + e][0][m]) for m in o] for e in range(n)])
                cache[key] = mpmath.det(M)
            return cache[key]
        psi = mpmath.mpf(0)
        for k in range(wl.n_det):
            psi += mpmath.mpf(wl.c[k]) * D(wl.det_up[k], 0, wl.n_up) * D(wl.det_dn[k], wl.n_up, wl.n_dn)
        assert float(mpmath.sign(psi)) == res.sign[w]
        assert abs(float(mpmath.log(abs(psi))) - res.logabs[w]) < 1e-13 * res.rs_psi[w]


def test_max_degree_equals_filtered_expansion():
    wl = make_config(2)
    from oracle.preprocess import occupied
    ref_u, ref_d = set(occupied(wl.det_up[0])), set(occupied(wl.det_dn[0]))
    deg_u = np.array([len(ref_u - set(occupied(d))) for d in wl.det_up])
    deg_d = np.array([len(ref_d - set(occupied(d))) for d in wl.det_dn])
    R = wl.R[:4]
    for dmax in (1, 2, 3):
        keep = (deg_u <= dmax) & (deg_d <= dmax)
        a = oracle.evaluate(wl, R, max_degree=np.full(4, dmax, np.int8), n_threads=2)
        b = oracle.evaluate(wl, R, c=wl.c[keep], det_up=wl.det_up[keep], det_dn=wl.det_dn[keep],
                            max_degree=None, n_threads=2)
        np.testing.assert_allclose(a.logabs, b.logabs, rtol=1e-13)
        np.testing.assert_allclose(a.gl, b.gl, rtol=1e-10, atol=1e-10)


def test_node_and_origin():
    wl = make_config(1)
    R = wl.R[:2].copy()
    R[0, 1] = R[0, 0]                # two up electrons at the same point -> Psi = 0
    R[1, 2] = 0.0                    # one electron exactly at the nucleus
    res = oracle.evaluate(wl, R, n_threads=1)
    assert res.sign[0] == 0.0 and res.logabs[0] == -np.inf and np.all(res.gl[0] == 0)
    assert np.isfinite(res.logabs[1]) and np.all(np.isfinite(res.gl[1]))
