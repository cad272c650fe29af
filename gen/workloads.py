"""Seeded synthetic workloads for the multideterminant evaluator.

This module only draws inputs: Gaussian-primitive orbitals, determinant
occupation lists written in the 64-bit-word input format, CI coefficients and
walker coordinates.  It holds none of the evaluation arithmetic, so both the
CPU oracle and the GPU library may consume what it produces.

Input format (the encoding of Sec. 2.1 "Encoding"): a spin determinant is
``n_int`` little-endian 64-bit words; bit ``b`` of word ``w`` set means that
molecular orbital ``64*w + b`` (0-based) is occupied.

Recipes (the paper's chlorine CIPSI wavefunctions are not available, so these
stand in for them; each config mirrors the shapes of Sec. 4 at the sizes of
the benchmark workloads):

* orbital m = sum_p coef[m,p] x^a y^b z^c exp(-alpha[m,p] r^2), centred at the
  origin, (a,b,c) uniform over the 10 monomials with a+b+c <= 2,
  alpha = exp(U(ln 0.1, ln 50)), coef ~ N(0,1), no normalisation; orbitals
  are then labelled in ascending order of their smallest exponent
  (diffuse first);
* reference spin determinant = orbitals 0..n_sigma-1; the other unique spin
  determinants are distinct random excitations of it, the degree uniform over
  the config's range, holes uniform among occupied orbitals, particles uniform
  among virtual orbitals;
* product 0 is (ref, ref) with c_0 = 0.95; the others are distinct uniform
  (i, j) pairs, |c_k| = A exp(-k/50) (tiny config) or A k^-1.2, random sign,
  with A chosen so that sum_k c_k^2 = 1;
* walkers: i.i.d. N(0, sigma^2) per coordinate;
* batched-uneven config: each walker draws a maximum excitation degree
  d_w ~ U{1..4}; it evaluates only products whose two spin determinants both
  have degree <= d_w.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional

import numpy as np


@dataclasses.dataclass
class Workload:
    name: str
    n_up: int
    n_dn: int
    n_mo: int
    n_prim: int
    pow_abc: np.ndarray      # int32 [n_mo][n_prim][3]
    alpha: np.ndarray        # f64   [n_mo][n_prim]
    coef: np.ndarray         # f64   [n_mo][n_prim]
    n_int: int
    det_up: np.ndarray       # uint64 [n_det][n_int]
    det_dn: np.ndarray       # uint64 [n_det][n_int]
    c: np.ndarray            # f64 [n_det]
    R: np.ndarray            # f64 [n_walk][n_up+n_dn][3]
    max_degree: Optional[np.ndarray] = None   # int8 [n_walk] or None
    # optional separate orbitals of the down electrons (same shapes)
    pow_abc_dn: Optional[np.ndarray] = None
    alpha_dn: Optional[np.ndarray] = None
    coef_dn: Optional[np.ndarray] = None

    @property
    def n_elec(self) -> int:
        return self.n_up + self.n_dn

    @property
    def n_det(self) -> int:
        return int(self.c.shape[0])

    @property
    def n_walk(self) -> int:
        return int(self.R.shape[0])


# shapes of the five benchmark workloads (index = config id)
CONFIGS = {
    1: dict(name="tiny", n_up=5, n_dn=5, n_mo=20, n_prim=3, n_uniq=50,
            degrees=(1, 2), n_det=500, coef_law="exp50", n_walk=8, sigma=1.5),
    2: dict(name="c2_1e4", n_up=9, n_dn=8, n_mo=60, n_prim=4, n_uniq=300,
            degrees=(1, 2, 3, 4), n_det=10_000, coef_law="pow1.2", n_walk=256,
            sigma=2.0),
    3: dict(name="c3_1e5", n_up=9, n_dn=8, n_mo=100, n_prim=4, n_uniq=1000,
            degrees=(1, 2, 3, 4), n_det=100_000, coef_law="pow1.2",
            n_walk=1024, sigma=2.0),
    4: dict(name="c4_uneven_7.5e5", n_up=9, n_dn=8, n_mo=120, n_prim=4,
            n_uniq=2500, degrees=(1, 2, 3, 4), n_det=750_000,
            coef_law="pow1.2", n_walk=4096, sigma=2.0, uneven=True),
    5: dict(name="c5_vmc", base=3, n_walk=2048),
}

MONOMIALS = [(a, b, c) for a in range(3) for b in range(3) for c in range(3)
             if a + b + c <= 2]
assert len(MONOMIALS) == 10


def encode(occ_lists, n_int: int) -> np.ndarray:
    """Occupied-orbital lists -> uint64 words (input format only)."""
    out = np.zeros((len(occ_lists), n_int), dtype=np.uint64)
    for k, occ in enumerate(occ_lists):
        for m in occ:
            out[k, m // 64] |= np.uint64(1) << np.uint64(m % 64)
    return out


def _orbitals(rng, n_mo, n_prim, relabel=True):
    mono = rng.integers(0, len(MONOMIALS), size=(n_mo, n_prim))
    pow_abc = np.array(MONOMIALS, dtype=np.int32)[mono]
    alpha = np.exp(rng.uniform(math.log(0.1), math.log(50.0), size=(n_mo, n_prim)))
    coef = rng.standard_normal((n_mo, n_prim))
    # label the orbitals diffuse-first (ascending smallest exponent), so the
    # reference determinant (orbitals 0..n-1) holds the most diffuse ones;
    # relabel=False keeps the order of the draw (a near-singular reference
    # at most walkers: the stress case of the conditioning fallback)
    if not relabel:
        return pow_abc.astype(np.int32), alpha, coef
    order = np.argsort(alpha.min(axis=1), kind="stable")
    return pow_abc[order].astype(np.int32), alpha[order], coef[order]


def _unique_dets(rng, n_sigma, n_mo, n_uniq, degrees):
    ref = tuple(range(n_sigma))
    seen = {ref}
    out = [ref]
    virt_all = np.arange(n_sigma, n_mo)
    while len(out) < n_uniq:
        s = int(rng.choice(degrees))
        holes = rng.choice(n_sigma, size=s, replace=False)
        parts = rng.choice(virt_all, size=s, replace=False)
        occ = sorted((set(ref) - set(int(h) for h in holes)) | set(int(p) for p in parts))
        t = tuple(occ)
        if t in seen:
            continue
        seen.add(t)
        out.append(t)
    return out


def _coefficients(rng, n_det, law):
    k = np.arange(1, n_det, dtype=np.float64)
    if law == "exp50":
        mag = np.exp(-k / 50.0)
    else:
        mag = k ** -1.2
    a = math.sqrt((1.0 - 0.95 ** 2) / float(np.sum(mag * mag))) if n_det > 1 else 0.0
    sign = np.where(rng.random(n_det - 1) < 0.5, -1.0, 1.0)
    return np.concatenate([[0.95], a * mag * sign])


def _pairs(rng, n_det, nu, nd):
    """k=0 -> (0,0); the rest distinct uniform pairs != (0,0)."""
    total = nu * nd
    if n_det > total:
        raise ValueError("more products than distinct pairs")
    flat = rng.choice(np.arange(1, total), size=n_det - 1, replace=False)
    flat = np.concatenate([[0], flat])
    return flat // nd, flat % nd


def make_config(cid: int, seed: Optional[int] = None, n_walk: Optional[int] = None,
                raw_orbital_order: bool = False) -> Workload:
    """Build benchmark workload ``cid`` (1..5) from SeedSequence(1000+cid);
    ``raw_orbital_order`` keeps the orbitals in the order drawn."""
    spec = dict(CONFIGS[cid])
    if "base" in spec:
        base = make_config(spec["base"], seed=seed, n_walk=n_walk or spec["n_walk"],
                           raw_orbital_order=raw_orbital_order)
        base.name = spec["name"]
        return base
    ss = np.random.SeedSequence(1000 + cid if seed is None else seed)
    s_orb, s_up, s_dn, s_pair, s_coef, s_walk, s_deg = (np.random.default_rng(s) for s in ss.spawn(7))
    n_up, n_dn, n_mo, n_prim = spec["n_up"], spec["n_dn"], spec["n_mo"], spec["n_prim"]
    pow_abc, alpha, coef = _orbitals(s_orb, n_mo, n_prim, relabel=not raw_orbital_order)
    n_int = (n_mo + 63) // 64
    ups = _unique_dets(s_up, n_up, n_mo, spec["n_uniq"], spec["degrees"])
    dns = _unique_dets(s_dn, n_dn, n_mo, spec["n_uniq"], spec["degrees"])
    ii, jj = _pairs(s_pair, spec["n_det"], len(ups), len(dns))
    c = _coefficients(s_coef, spec["n_det"], spec["coef_law"])
    up_words = encode(ups, n_int)
    dn_words = encode(dns, n_int)
    W = spec["n_walk"] if n_walk is None else n_walk
    R = s_walk.normal(0.0, spec["sigma"], size=(W, n_up + n_dn, 3))
    md = None
    if spec.get("uneven"):
        md = s_deg.integers(1, 5, size=W).astype(np.int8)
    return Workload(name=spec["name"], n_up=n_up, n_dn=n_dn, n_mo=n_mo, n_prim=n_prim,
                    pow_abc=pow_abc, alpha=alpha, coef=coef, n_int=n_int,
                    det_up=np.ascontiguousarray(up_words[ii]),
                    det_dn=np.ascontiguousarray(dn_words[jj]),
                    c=c, R=R, max_degree=md)


def make_custom(n_up, n_dn, n_mo, n_prim, n_uniq_up, n_uniq_dn, degrees, n_det,
                n_walk, sigma=2.0, seed=0, coef_law="pow1.2", uneven=False,
                alpha_range=(0.1, 50.0)) -> Workload:
    """Same recipe with free shapes (used for ragged-size parity cases)."""
    ss = np.random.SeedSequence(seed)
    s_orb, s_up, s_dn, s_pair, s_coef, s_walk, s_deg = (np.random.default_rng(s) for s in ss.spawn(7))
    mono = s_orb.integers(0, len(MONOMIALS), size=(n_mo, n_prim))
    pow_abc = np.array(MONOMIALS, dtype=np.int32)[mono]
    alpha = np.exp(s_orb.uniform(math.log(alpha_range[0]), math.log(alpha_range[1]),
                                 size=(n_mo, n_prim)))
    coef = s_orb.standard_normal((n_mo, n_prim))
    order = np.argsort(alpha.min(axis=1), kind="stable")
    pow_abc, alpha, coef = pow_abc[order], alpha[order], coef[order]
    n_int = (n_mo + 63) // 64
    ups = _unique_dets(s_up, n_up, n_mo, n_uniq_up, degrees)
    dns = _unique_dets(s_dn, n_dn, n_mo, n_uniq_dn, degrees)
    ii, jj = _pairs(s_pair, n_det, len(ups), len(dns))
    c = _coefficients(s_coef, n_det, coef_law)
    R = s_walk.normal(0.0, sigma, size=(n_walk, n_up + n_dn, 3))
    md = s_deg.integers(1, 5, size=n_walk).astype(np.int8) if uneven else None
    return Workload(name=f"custom{seed}", n_up=n_up, n_dn=n_dn, n_mo=n_mo, n_prim=n_prim,
                    pow_abc=pow_abc.astype(np.int32), alpha=alpha, coef=coef, n_int=n_int,
                    det_up=np.ascontiguousarray(encode(ups, n_int)[ii]),
                    det_dn=np.ascontiguousarray(encode(dns, n_int)[jj]),
                    c=c, R=R, max_degree=md)


def with_down_orbitals(wl: Workload, seed: int = 1) -> Workload:
    """The same workload with a second, independently drawn orbital set for
    the down electrons (same monomials, other exponents and coefficients)."""
    rng = np.random.default_rng(np.random.SeedSequence(seed))
    alpha = wl.alpha * np.exp(rng.uniform(-0.3, 0.3, size=wl.alpha.shape))
    coef = rng.standard_normal(wl.coef.shape)
    return dataclasses.replace(wl, pow_abc_dn=wl.pow_abc.copy(), alpha_dn=alpha, coef_dn=coef)


def make_helium(n_walk: int, seed: int = 0, sigma: float = 0.8) -> Workload:
    """Two electrons (one per spin) in one nodeless s orbital, a sum of two
    Gaussians, as a single determinant: the helium atom (nuclear charge 2)
    for the diffusion Monte Carlo checks.  Walkers start normal around the
    nucleus."""
    rng = np.random.default_rng(np.random.SeedSequence(seed))
    pow_abc = np.zeros((1, 2, 3), dtype=np.int32)
    alpha = np.array([[0.45, 2.2]])
    coef = np.array([[1.0, 0.6]])
    det = encode([[0]], 1)
    R = rng.normal(0.0, sigma, size=(n_walk, 2, 3))
    return Workload(name="helium", n_up=1, n_dn=1, n_mo=1, n_prim=2, pow_abc=pow_abc,
                    alpha=alpha, coef=coef, n_int=1, det_up=det.copy(), det_dn=det.copy(),
                    c=np.array([1.0]), R=R, max_degree=None)


def walker_pool(wl: Workload, n_pool: int, seed: int = 7, sigma: float = 2.0) -> np.ndarray:
    """Extra walker sets of the same distribution (rotated per timed step)."""
    rng = np.random.default_rng(np.random.SeedSequence(seed))
    return rng.normal(0.0, sigma, size=(n_pool,) + wl.R.shape)


def mlp_init(n_in: int, n_hid: int, n_out: int, seed: int = 0, out_scale: float = 0.05) -> np.ndarray:
    """Initial parameters of the proposal network (flat FP32, layout
    [W1, b1, W2, b2, W3, b3]): uniform +-1/sqrt(fan_in) hidden layers, a small
    output layer, zero biases except the log-step bias (ln 0.3, a modest
    initial step)."""
    rng = np.random.default_rng(np.random.SeedSequence(seed))
    W1 = rng.uniform(-1, 1, (n_in, n_hid)) / math.sqrt(n_in)
    W2 = rng.uniform(-1, 1, (n_hid, n_hid)) / math.sqrt(n_hid)
    W3 = rng.uniform(-1, 1, (n_hid, n_out)) * out_scale / math.sqrt(n_hid)
    b3 = np.zeros(n_out)
    n_e = n_out // 4
    b3[3 * n_e:] = math.log(0.3)
    parts = [W1, np.zeros(n_hid), W2, np.zeros(n_hid), W3, b3]
    return np.concatenate([p.ravel() for p in parts]).astype(np.float32)
