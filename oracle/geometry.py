"""Oracle node sets for the image-enhanced MFS discretisation (test infrastructure).

Everything here is written from the paper:
  * proxy Stokeslets on a concentric sphere of radius R_p, collocation nodes
    on the surface (Section 2.1);
  * accumulation points of repeated Kelvin reflections, eq. (acc_points),
    their distance R_acc(delta), eq. (Racc), and the critical gap delta*,
    eq. (deltastar) (Section 2.3);
  * image-line nodes t_j, eqs. (line_points)-(tj) (Section 2.3);
  * two collocation caps per contact, eqs. (colloc_nbr)-(thetacap)
    (Section 5.1), read as cos(theta_j) = 1 - j (1 - cos beta) / M_cap
    because the printed form does not produce caps of half-angle beta;
  * left weights = local area per collocation node (Remark left-precond);
  * per-sphere counts N_S, N_R, N_D and M, eq. (Mest) (Section 5.1).

Point sets: the paper uses spherical designs, which are not available; the
Fibonacci spiral cos(theta_j) = 1 - (2j-1)/n, phi_j = 2 pi j / Phi mod 2 pi,
j = 1..n, stands in for them (the paper itself uses Fibonacci grids for the
caps).

Conventions shared with any implementation that exchanges arrays with this
oracle (they are a data contract, not code):
  * targets of sphere k: base nodes, then for each contact (neighbours in
    increasing index) the beta_1 cap then the beta_2 cap;
  * sources are packed globally in four blocks, each sphere-major: every
    proxy Stokeslet, then every image Stokeslet (contact by contact), then
    every rotlet, then every potential dipole;
  * the local source order of sphere k (the columns of its self block) is
    its proxy Stokeslets, image Stokeslets, rotlets, dipoles;
  * vectors are node-major: entry 3 i + c is component c of node i.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

GOLDEN = (1.0 + math.sqrt(5.0)) / 2.0
KIND_S, KIND_R, KIND_D = 0, 1, 2
# packing blocks: proxy Stokeslets, image Stokeslets, rotlets, dipoles
BLOCK_KIND = (KIND_S, KIND_S, KIND_R, KIND_D)


@dataclass
class Params:
    n_proxy: int = 600
    proxy_radius: float = 0.7          # R_p, in radii
    n_colloc_base: int = 780
    n_image: int = 20                  # < 0: adaptive rule eq. (image_est)
    kinds: str = "SRD"                 # kinds placed at image nodes
    image_offset: float = 0.05         # Delta in eq. (tj)
    image_gap_cutoff: float = 0.2      # pairs closer than this get images
    near_gap_cutoff: float = 0.2
    cap_alpha: tuple = (6, 6)
    cap_beta: tuple = (math.pi / 5.0, math.pi / 60.0)
    left_weights: bool = True
    trunc_rel: float = 5e-12
    mu: float = 1.0
    n_check_base: int = 500


# -- closed forms ----------------------------------------------------------

def fibonacci_sphere(n: int, half_shift: bool = False) -> np.ndarray:
    """Unit vectors of the n-point Fibonacci spiral.  With half_shift the
    azimuth uses j + 1/2, which interleaves a second set (check points)."""
    j = np.arange(1, n + 1, dtype=np.float64)
    cos_t = 1.0 - (2.0 * j - 1.0) / n
    sin_t = np.sqrt(np.maximum(0.0, 1.0 - cos_t * cos_t))
    jj = j + (0.5 if half_shift else 0.0)
    phi = np.mod(2.0 * math.pi * jj / GOLDEN, 2.0 * math.pi)
    return np.stack([sin_t * np.cos(phi), sin_t * np.sin(phi), cos_t], 1)


def r_acc(delta: float) -> float:
    """Distance from the centre to the image accumulation point, eq. (Racc)."""
    return 1.0 + delta / 2.0 - math.sqrt(delta + delta * delta / 4.0)


def delta_star(Rp: float) -> float:
    """Critical gap where R_acc equals R_p, eq. (deltastar)."""
    return (1.0 - Rp) ** 2 / Rp


def kelvin_reflect(x: np.ndarray, c: np.ndarray, a: float = 1.0) -> np.ndarray:
    """Image of x in the sphere of centre c and radius a, eq. (reflect)
    (stated there for a = 1)."""
    d = x - c
    return c + a * a * d / float(d @ d)


def accumulation_points(c1: np.ndarray, c2: np.ndarray, a: float = 1.0):
    """Fixed points of repeated reflection, eq. (acc_points); gap in radii."""
    dist = float(np.linalg.norm(c2 - c1))
    delta = dist / a - 2.0
    e = (c2 - c1) / dist
    mid = 0.5 * (c1 + c2)
    s = a * math.sqrt(delta + delta * delta / 4.0)
    return mid - s * e, mid + s * e


def image_t(delta: float, Rp: float, n_im: int, Delta: float) -> np.ndarray:
    """Image-node radii t_j, j = 1..n_im, eq. (tj) (in radii)."""
    j = np.arange(1, n_im + 1, dtype=np.float64)
    t0 = Rp * (1.0 + Delta)
    return t0 + (r_acc(delta) - t0) * np.cos((j - 1.0) * math.pi / (2.0 * n_im))


def n_image_rule(delta: float) -> int:
    """Adaptive image count, eq. (image_est)."""
    if delta < 0.15:
        return int(math.ceil(-8.72 * math.log10(delta) - 6.15))
    return 0


def axis_frame(e: np.ndarray):
    """Two unit vectors completing e to a right-handed frame (the cap azimuth
    origin, which the paper leaves open)."""
    z = np.array([0.0, 0.0, 1.0])
    e1 = np.cross(e, z)
    if np.linalg.norm(e1) < 0.1:
        e1 = np.cross(e, np.array([1.0, 0.0, 0.0]))
    e1 = e1 / np.linalg.norm(e1)
    e2 = np.cross(e, e1)
    return e1, e2


def cap_local(m: int, beta: float, half_shift: bool = False) -> np.ndarray:
    """(cos theta, sin theta cos phi, sin theta sin phi) for an m-point
    Fibonacci cap of half-angle beta around the local pole."""
    j = np.arange(1, m + 1, dtype=np.float64)
    jt = j - (0.5 if half_shift else 0.0)
    cos_t = 1.0 - jt * (1.0 - math.cos(beta)) / m
    sin_t = np.sqrt(np.maximum(0.0, 1.0 - cos_t * cos_t))
    jp = j + (0.5 if half_shift else 0.0)
    phi = np.mod(2.0 * math.pi * jp / GOLDEN, 2.0 * math.pi)
    return np.stack([cos_t, sin_t * np.cos(phi), sin_t * np.sin(phi)], 1)


def cap_points(c, a, e, m, beta, half_shift=False) -> np.ndarray:
    e1, e2 = axis_frame(e)
    loc = cap_local(m, beta, half_shift)
    return c + a * (loc[:, :1] * e + loc[:, 1:2] * e1 + loc[:, 2:3] * e2)


# -- the discretised problem ----------------------------------------------

@dataclass
class Contact:
    other: int
    gap: float            # in radii
    axis: np.ndarray      # unit vector towards the neighbour
    n_im: int


@dataclass
class Geometry:
    params: Params
    centers: np.ndarray
    radius: float
    contacts: list                     # per sphere: list[Contact]
    targets: np.ndarray                # (T, 3)
    target_sphere: np.ndarray          # (T,)
    target_weight: np.ndarray          # (T,) area weights w_i
    target_offsets: np.ndarray         # (P+1,)
    src_pos: np.ndarray                # (S, 3), packed by kind
    src_kind: np.ndarray               # (S,)
    src_sphere: np.ndarray             # (S,)
    kind_offsets: np.ndarray           # (4, P+1): sphere ranges in each packing block
    local_sources: list                # per sphere: packed indices, local order
    check: np.ndarray                  # (C, 3) residual check points
    check_sphere: np.ndarray
    check_offsets: np.ndarray
    n_kind: np.ndarray = field(default_factory=lambda: np.zeros(3, np.int64))
    n_block: np.ndarray = field(default_factory=lambda: np.zeros(4, np.int64))

    @property
    def P(self):
        return int(self.centers.shape[0])

    @property
    def T(self):
        return int(self.targets.shape[0])

    @property
    def S(self):
        return int(self.src_pos.shape[0])

    def M(self, k):
        return int(self.target_offsets[k + 1] - self.target_offsets[k])

    def Nk(self, k):
        return len(self.local_sources[k])

    def contact_free(self, k):
        return len(self.contacts[k]) == 0


def find_contacts(centers, a, prm: Params):
    P = centers.shape[0]
    out = [[] for _ in range(P)]
    for k in range(P):
        for kk in range(P):
            if kk == k:
                continue
            d = centers[kk] - centers[k]
            dist = float(np.linalg.norm(d))
            gap = dist / a - 2.0
            if gap <= 0.0:
                raise ValueError(f"spheres {k} and {kk} overlap")
            if gap < prm.image_gap_cutoff:
                n_im = prm.n_image if prm.n_image >= 0 else n_image_rule(gap)
                if n_im > 0:
                    out[k].append(Contact(kk, gap, d / dist, n_im))
    return out


def build(centers, radius: float, prm: Params | None = None) -> Geometry:
    """Assemble every node set of the discretisation (see module docstring)."""
    prm = prm or Params()
    centers = np.asarray(centers, np.float64)
    a = float(radius)
    P = centers.shape[0]
    contacts = find_contacts(centers, a, prm)
    proxy = fibonacci_sphere(prm.n_proxy) * (prm.proxy_radius * a)
    base = fibonacci_sphere(prm.n_colloc_base) * a
    chk = fibonacci_sphere(prm.n_check_base, half_shift=True) * a
    w_base = 4.0 * math.pi * a * a / prm.n_colloc_base

    tg, tg_s, tg_w, toff = [], [], [], [0]
    ck, ck_s, coff = [], [], [0]
    per_block = [[], [], [], []]
    for k in range(P):
        c = centers[k]
        blocks = [c + base]
        wts = [np.full(prm.n_colloc_base, w_base)]
        cblocks = [c + chk]
        s_img, r_pos, d_pos = [], [], []
        for ct in contacts[k]:
            t = image_t(ct.gap, prm.proxy_radius, ct.n_im, prm.image_offset)
            line = c + a * t[:, None] * ct.axis[None, :]
            if "S" in prm.kinds:
                s_img.append(line)
            if "R" in prm.kinds:
                r_pos.append(line)
            if "D" in prm.kinds:
                d_pos.append(line)
            for alpha, beta in zip(prm.cap_alpha, prm.cap_beta):
                m = int(alpha * 3 * ct.n_im)
                blocks.append(cap_points(c, a, ct.axis, m, beta))
                wts.append(np.full(m, 2.0 * math.pi * a * a * (1.0 - math.cos(beta)) / m))
                cblocks.append(cap_points(c, a, ct.axis, m, beta, half_shift=True))
        X = np.concatenate(blocks)
        tg.append(X)
        tg_s.append(np.full(len(X), k))
        tg_w.append(np.concatenate(wts))
        toff.append(toff[-1] + len(X))
        C = np.concatenate(cblocks)
        ck.append(C)
        ck_s.append(np.full(len(C), k))
        coff.append(coff[-1] + len(C))
        empty = np.zeros((0, 3))
        per_block[0].append(c + proxy)
        per_block[1].append(np.concatenate(s_img) if s_img else empty)
        per_block[2].append(np.concatenate(r_pos) if r_pos else empty)
        per_block[3].append(np.concatenate(d_pos) if d_pos else empty)

    kind_off = np.zeros((4, P + 1), np.int64)
    pos_all, kind_all, sph_all = [], [], []
    base_idx = 0
    n_block = np.zeros(4, np.int64)
    for blk in range(4):
        kind_off[blk, 0] = base_idx
        for k in range(P):
            arr = per_block[blk][k]
            pos_all.append(arr)
            kind_all.append(np.full(len(arr), BLOCK_KIND[blk]))
            sph_all.append(np.full(len(arr), k))
            base_idx += len(arr)
            kind_off[blk, k + 1] = base_idx
        n_block[blk] = kind_off[blk, P] - kind_off[blk, 0]
    n_kind = np.array([n_block[0] + n_block[1], n_block[2], n_block[3]], np.int64)
    local = []
    for k in range(P):
        idx = np.concatenate([np.arange(kind_off[b, k], kind_off[b, k + 1]) for b in range(4)])
        local.append(idx.astype(np.int64))
    return Geometry(
        params=prm, centers=centers, radius=a, contacts=contacts,
        targets=np.concatenate(tg), target_sphere=np.concatenate(tg_s),
        target_weight=np.concatenate(tg_w), target_offsets=np.asarray(toff, np.int64),
        src_pos=np.concatenate(pos_all), src_kind=np.concatenate(kind_all).astype(np.int32),
        src_sphere=np.concatenate(sph_all).astype(np.int32), kind_offsets=kind_off,
        local_sources=local, check=np.concatenate(ck),
        check_sphere=np.concatenate(ck_s), check_offsets=np.asarray(coff, np.int64),
        n_kind=n_kind, n_block=n_block)


def m_estimate(n_base: int, n_ims) -> int:
    """Collocation count of a sphere, eq. (Mest), with the base count given."""
    return int(n_base + 2 * 6 * sum(3 * n for n in n_ims))
