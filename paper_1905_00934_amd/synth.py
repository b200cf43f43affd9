"""Seeded synthetic inputs: a dual-energy scanner simulator.

This module produces every input that both the reconstruction library and
the oracle consume, and nothing else: the energy grid, two tungsten-like
spectra, the Compton (Klein-Nishina) and photoelectric energy multipliers of
the attenuation model (Sec. 1, Eq. (1)), luggage-like phantoms made of
ellipses and rectangles, their exact (analytic) line integrals, and Poisson
photon counts drawn from the polychromatic Beer-Lambert law (Sec. 1, Eq. (2)).

It holds none of the reconstruction's arithmetic: no projector, no
decomposition, no ADMM step.  The line integrals are closed-form chord
lengths through the shapes, so the simulated data are not produced by the
discrete projector that the reconstruction inverts.

Geometry convention (shared by the data model, the reconstruction library and
the oracle, each of which implements it on its own):
  * pixel (j, i) of an ny-by-nx image, stored row-major, has its centre at
    x_i = (i - (nx-1)/2) * pixel_cm,  y_j = (j - (ny-1)/2) * pixel_cm;
  * view v is at angle theta_v = angle0 + v * span / n_views;
  * parallel beam: ray (v, b) is the line {p : p . (cos t, sin t) = t_b},
    t_b = (b - (n_det-1)/2 + det_offset) * det_cm, direction (-sin t, cos t);
  * fan beam, flat detector: source s = R_so (cos t, sin t), bin b at
    -(R_sd - R_so)(cos t, sin t) + u_b (-sin t, cos t),
    u_b = (b - (n_det-1)/2 + det_offset) * det_cm; the ray runs from s to the bin.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

ELECTRON_REST_KEV = 510.998_95

# -----------------------------------------------------------------------------
# Energy grid, attenuation multipliers, spectra
# -----------------------------------------------------------------------------


def energy_grid(e_min: float = 20.0, e_max: float = 130.0, step: float = 1.0) -> np.ndarray:
    """Energies in keV at the centres of the spectral bins (1 keV bins, 20-130 keV)."""
    n = int(round((e_max - e_min) / step)) + 1
    return e_min + step * np.arange(n, dtype=np.float64)


def klein_nishina(energy_kev) -> np.ndarray:
    """Total Klein-Nishina cross-section per electron divided by 2*pi*r_e^2.

    This is the energy dependence of Compton scattering used as f_KN(E) in the
    attenuation model of Sec. 1, Eq. (1).  It tends to 4/3 (Thomson) as E -> 0.
    """
    e = np.asarray(energy_kev, dtype=np.float64)
    a = e / ELECTRON_REST_KEV
    l2a = np.log1p(2.0 * a)
    return ((1.0 + a) / a**2 * (2.0 * (1.0 + a) / (1.0 + 2.0 * a) - l2a / a)
            + l2a / (2.0 * a) - (1.0 + 3.0 * a) / (1.0 + 2.0 * a) ** 2)


def photoelectric(energy_kev, e_ref: float = 60.0) -> np.ndarray:
    """Photoelectric energy multiplier f_p(E) = (E_ref / E)^3 (Sec. 1: cubic decay)."""
    e = np.asarray(energy_kev, dtype=np.float64)
    return (e_ref / e) ** 3


# Two-basis (Compton, photoelectric) coefficients in 1/cm of the materials the
# phantoms are built from, for f_KN as above and f_p with E_ref = 60 keV.
WATER = (0.18, 0.018)
ALUMINIUM = (0.42, 0.25)


def tungsten_spectrum(kvp: float, energy_kev: np.ndarray, al_filter_cm: float = 0.25) -> np.ndarray:
    """Photon-count spectrum of a tungsten-anode tube (Kramers law, Al filtration, K lines).

    Unnormalised; zero at and above kVp.  The continuum is (kVp - E)/E photons per
    keV, filtered by al_filter_cm of aluminium; the tungsten K lines at 58, 59 and
    67 keV are added when kVp exceeds the K edge (69.5 keV).
    """
    e = np.asarray(energy_kev, dtype=np.float64)
    mu_al = ALUMINIUM[0] * klein_nishina(e) + ALUMINIUM[1] * photoelectric(e)
    cont = np.maximum(kvp - e, 0.0) / e * np.exp(-al_filter_cm * mu_al)
    s = cont.copy()
    if kvp > 69.5:
        ref = float(np.interp(59.0, e, cont))
        for line_kev, amp in ((58.0, 0.6), (59.0, 1.0), (67.0, 0.35)):
            k = int(np.argmin(np.abs(e - line_kev)))
            if abs(e[k] - line_kev) < 0.5:
                s[k] += amp * 2.0 * ref
    s[e >= kvp] = 0.0
    return s


@dataclass
class Spectra:
    """The spectral inputs of the forward model (Sec. 3.1, Eq. (3))."""
    energy_kev: np.ndarray
    s_high: np.ndarray
    s_low: np.ndarray
    f_kn: np.ndarray
    f_p: np.ndarray

    @property
    def n_bins(self) -> int:
        return int(self.energy_kev.size)


def default_spectra(kvp_high: float = 130.0, kvp_low: float = 95.0) -> Spectra:
    e = energy_grid()
    return Spectra(e, tungsten_spectrum(kvp_high, e), tungsten_spectrum(kvp_low, e),
                   klein_nishina(e), photoelectric(e))


def monochromatic_spectra(e_high: float, e_low: float) -> Spectra:
    """Two single-line spectra on the default grid (for the linear special case)."""
    e = energy_grid()
    sh = np.zeros_like(e)
    sl = np.zeros_like(e)
    sh[int(np.argmin(np.abs(e - e_high)))] = 1.0
    sl[int(np.argmin(np.abs(e - e_low)))] = 1.0
    return Spectra(e, sh, sl, klein_nishina(e), photoelectric(e))


# -----------------------------------------------------------------------------
# Geometry
# -----------------------------------------------------------------------------


def geometry(kind: str, nx: int, ny: int, pixel_cm: float, n_views: int, n_det: int,
             det_cm: float, det_offset: float = 0.0, src_iso_cm: float = 0.0,
             src_det_cm: float = 0.0, angle0: float = 0.0, span: float | None = None) -> dict:
    if kind not in ("parallel", "fan"):
        raise ValueError(kind)
    if span is None:
        span = math.pi if kind == "parallel" else 2.0 * math.pi
    return dict(kind=kind, nx=int(nx), ny=int(ny), pixel_cm=float(pixel_cm),
                n_views=int(n_views), n_det=int(n_det), det_cm=float(det_cm),
                det_offset=float(det_offset), src_iso_cm=float(src_iso_cm),
                src_det_cm=float(src_det_cm), angle0=float(angle0), span=float(span))


def fan_geometry_fov(n: int, n_views: int, n_det: int, fov_cm: float = 51.2,
                     src_iso_cm: float = 54.0, src_det_cm: float = 95.0) -> dict:
    """Fan-beam scanner whose flat detector covers the circle circumscribing the FOV square."""
    r_circ = fov_cm / math.sqrt(2.0)
    half = src_det_cm * math.tan(math.asin(r_circ / src_iso_cm))
    return geometry("fan", n, n, fov_cm / n, n_views, n_det, 2.0 * half / n_det,
                    src_iso_cm=src_iso_cm, src_det_cm=src_det_cm)


def ray_lines(geom: dict):
    """Origin and unit direction of every ray, shapes [V, D, 2] (data model only)."""
    V, D = geom["n_views"], geom["n_det"]
    th = geom["angle0"] + np.arange(V) * geom["span"] / V
    c, s = np.cos(th)[:, None], np.sin(th)[:, None]
    u = (np.arange(D) - (D - 1) / 2.0 + geom["det_offset"]) * geom["det_cm"]
    u = u[None, :]
    if geom["kind"] == "parallel":
        ox, oy = u * c, u * s
        dx, dy = -s + 0 * u, c + 0 * u
    else:
        rso, rsd = geom["src_iso_cm"], geom["src_det_cm"]
        sx, sy = rso * c, rso * s
        qx = -(rsd - rso) * c - u * s
        qy = -(rsd - rso) * s + u * c
        dx, dy = qx - sx, qy - sy
        nrm = np.hypot(dx, dy)
        dx, dy = dx / nrm, dy / nrm
        ox, oy = sx + 0 * u, sy + 0 * u
    return np.stack([ox, oy], -1), np.stack([dx, dy], -1)


# -----------------------------------------------------------------------------
# Phantoms
# -----------------------------------------------------------------------------


@dataclass
class Shape:
    kind: str          # "ellipse" or "rect"
    cx: float
    cy: float
    ax: float          # semi-axis / half-width along the shape's own x
    ay: float
    rot: float         # rotation of the shape's x axis, radians
    xc: float          # Compton coefficient added inside, 1/cm
    xp: float          # photoelectric coefficient added inside, 1/cm

    def inside(self, x, y):
        c, s = math.cos(self.rot), math.sin(self.rot)
        u = (x - self.cx) * c + (y - self.cy) * s
        v = -(x - self.cx) * s + (y - self.cy) * c
        if self.kind == "ellipse":
            return (u / self.ax) ** 2 + (v / self.ay) ** 2 <= 1.0
        return (np.abs(u) <= self.ax) & (np.abs(v) <= self.ay)

    def chord(self, origin, direction):
        """Exact length of the intersection of each line with the shape.

        Lines farther from the centre than the shape's circumradius miss it; the
        exact formula runs on the others only.
        """
        r = max(self.ax, self.ay) if self.kind == "ellipse" else math.hypot(self.ax, self.ay)
        ox, oy = origin[..., 0] - self.cx, origin[..., 1] - self.cy
        dist = np.abs(ox * direction[..., 1] - oy * direction[..., 0]) / np.hypot(
            direction[..., 0], direction[..., 1])
        hit = dist <= r * (1.0 + 1e-9)
        out = np.zeros(origin.shape[:-1])
        if hit.any():
            out[hit] = self._chord(origin[hit], direction[hit])
        return out

    def _chord(self, origin, direction):
        c, s = math.cos(self.rot), math.sin(self.rot)
        px = (origin[..., 0] - self.cx) * c + (origin[..., 1] - self.cy) * s
        py = -(origin[..., 0] - self.cx) * s + (origin[..., 1] - self.cy) * c
        dx = direction[..., 0] * c + direction[..., 1] * s
        dy = -direction[..., 0] * s + direction[..., 1] * c
        if self.kind == "ellipse":
            px, py, dx, dy = px / self.ax, py / self.ay, dx / self.ax, dy / self.ay
            qa = dx * dx + dy * dy
            qb = px * dx + py * dy
            qc = px * px + py * py - 1.0
            disc = qb * qb - qa * qc
            return np.where(disc > 0.0, 2.0 * np.sqrt(np.maximum(disc, 0.0)) / qa, 0.0)
        lo = np.full(px.shape, -np.inf)
        hi = np.full(px.shape, np.inf)
        for p, d, h in ((px, dx, self.ax), (py, dy, self.ay)):
            with np.errstate(divide="ignore", invalid="ignore"):
                t1 = (-h - p) / d
                t2 = (h - p) / d
            par = d == 0.0
            tlo = np.where(par, np.where(np.abs(p) <= h, -np.inf, np.inf), np.minimum(t1, t2))
            thi = np.where(par, np.where(np.abs(p) <= h, np.inf, -np.inf), np.maximum(t1, t2))
            lo = np.maximum(lo, tlo)
            hi = np.minimum(hi, thi)
        return np.maximum(hi - lo, 0.0)

    def bbox(self):
        c, s = abs(math.cos(self.rot)), abs(math.sin(self.rot))
        if self.kind == "ellipse":
            hx = math.sqrt((self.ax * c) ** 2 + (self.ay * s) ** 2)
            hy = math.sqrt((self.ax * s) ** 2 + (self.ay * c) ** 2)
        else:
            hx = self.ax * c + self.ay * s
            hy = self.ax * s + self.ay * c
        return self.cx - hx, self.cx + hx, self.cy - hy, self.cy + hy


@dataclass
class Phantom:
    shapes: list = field(default_factory=list)

    def line_integrals(self, geom: dict):
        """Analytic (a_c, a_p) = integrals of x_c, x_p along every ray, [V, D] each."""
        o, d = ray_lines(geom)
        ac = np.zeros(o.shape[:2])
        ap = np.zeros(o.shape[:2])
        for sh in self.shapes:
            ln = sh.chord(o, d)
            ac += sh.xc * ln
            ap += sh.xp * ln
        return ac, ap

    def image(self, nx: int, ny: int, pixel_cm: float, supersample: int = 8):
        """Area-weighted ground truth (x_c, x_p) on the pixel grid, [ny, nx] each."""
        xc = np.zeros((ny, nx))
        xp = np.zeros((ny, nx))
        S = supersample
        off = ((np.arange(S) + 0.5) / S - 0.5) * pixel_cm
        for sh in self.shapes:
            x0, x1, y0, y1 = sh.bbox()
            i0 = max(int(math.floor(x0 / pixel_cm + (nx - 1) / 2.0)) - 1, 0)
            i1 = min(int(math.ceil(x1 / pixel_cm + (nx - 1) / 2.0)) + 1, nx - 1)
            j0 = max(int(math.floor(y0 / pixel_cm + (ny - 1) / 2.0)) - 1, 0)
            j1 = min(int(math.ceil(y1 / pixel_cm + (ny - 1) / 2.0)) + 1, ny - 1)
            if i1 < i0 or j1 < j0:
                continue
            xs = (np.arange(i0, i1 + 1) - (nx - 1) / 2.0) * pixel_cm
            ys = (np.arange(j0, j1 + 1) - (ny - 1) / 2.0) * pixel_cm
            X = xs[None, :, None, None] + off[None, None, None, :]
            Y = ys[:, None, None, None] + off[None, None, :, None]
            frac = sh.inside(X, Y).mean(axis=(2, 3))
            xc[j0:j1 + 1, i0:i1 + 1] += sh.xc * frac
            xp[j0:j1 + 1, i0:i1 + 1] += sh.xp * frac
        return xc, xp


def tiny_phantom(seed: int = 0, fov_cm: float = 32.0) -> Phantom:
    """Three disjoint ellipses with x_c in [0.15, 0.45] and x_p in [0, 0.02]."""
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([seed, 7001])))
    shapes = []
    placed = []
    while len(shapes) < 3:
        ax, ay = rng.uniform(2.0, 5.5, 2)
        r = max(ax, ay)
        ang = rng.uniform(0, 2 * math.pi)
        rad = rng.uniform(0, 0.5 * fov_cm - 2.0 - r)
        cx, cy = rad * math.cos(ang), rad * math.sin(ang)
        if any(math.hypot(cx - px, cy - py) < r + pr + 0.3 for px, py, pr in placed):
            continue
        placed.append((cx, cy, r))
        shapes.append(Shape("ellipse", cx, cy, ax, ay, rng.uniform(0, math.pi),
                            rng.uniform(0.15, 0.45), rng.uniform(0.0, 0.02)))
    return Phantom(shapes)


def luggage_phantom(seed: int, n_objects: int = 30, n_steel: int = 2,
                    fov_cm: float = 51.2) -> Phantom:
    """Bag shell plus non-overlapping organics, water, aluminium and steel inserts.

    The shell is an elliptical plastic annulus 0.3 cm thick (outer ellipse minus
    inner ellipse); objects are half ellipses, half rectangles, placed inside it
    without overlap of their bounding circles.  n_objects counts the steel inserts.
    """
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([seed, 7002])))
    scale = fov_cm / 51.2
    A = 22.0 * scale * rng.uniform(0.93, 1.03)
    B = 16.0 * scale * rng.uniform(0.93, 1.07)
    rot = rng.uniform(0, math.pi)
    bcx, bcy = rng.uniform(-1.0, 1.0, 2) * scale
    plastic = (0.20, 0.006)
    shapes = [Shape("ellipse", bcx, bcy, A, B, rot, *plastic),
              Shape("ellipse", bcx, bcy, A - 0.3, B - 0.3, rot, -plastic[0], -plastic[1])]
    inner_a, inner_b = A - 0.6, B - 0.6
    cr, sr = math.cos(rot), math.sin(rot)

    def fits(cx, cy, r):
        u = (cx - bcx) * cr + (cy - bcy) * sr
        v = -(cx - bcx) * sr + (cy - bcy) * cr
        ea, eb = inner_a - r, inner_b - r
        return ea > 0 and eb > 0 and (u / ea) ** 2 + (v / eb) ** 2 <= 1.0

    placed = []
    kinds = ["steel"] * n_steel
    for _ in range(max(n_objects - n_steel, 0)):
        t = rng.uniform()
        kinds.append("organic" if t < 0.60 else ("water" if t < 0.85 else "aluminium"))
    for kind in kinds:
        steel = kind == "steel"
        lo, hi = (0.3, 1.0) if steel else (0.5, 5.0)
        ax, ay = rng.uniform(lo, hi, 2) * scale
        shape_kind = "ellipse" if rng.uniform() < 0.5 else "rect"
        srot = rng.uniform(0, math.pi)
        if kind == "organic":
            mat = (rng.uniform(0.15, 0.25), rng.uniform(0.002, 0.02))
        elif kind == "water":
            mat = WATER
        elif kind == "aluminium":
            mat = ALUMINIUM
        else:
            mat = (rng.uniform(1.8, 2.2), rng.uniform(4.0, 6.0))
        ok = False
        for _attempt in range(12):
            r = math.hypot(ax, ay) if shape_kind == "rect" else max(ax, ay)
            for _try in range(60):
                cx = bcx + rng.uniform(-inner_a, inner_a)
                cy = bcy + rng.uniform(-inner_a, inner_a)
                if fits(cx, cy, r) and all(math.hypot(cx - px, cy - py) >= r + pr + 0.1
                                           for px, py, pr in placed):
                    ok = True
                    break
            if ok:
                break
            ax, ay = 0.8 * ax, 0.8 * ay
        if not ok:
            continue
        placed.append((cx, cy, r))
        shapes.append(Shape(shape_kind, cx, cy, ax, ay, srot, mat[0], mat[1]))
    return Phantom(shapes)


# -----------------------------------------------------------------------------
# Measurements
# -----------------------------------------------------------------------------


def expected_counts(spec: Spectra, a_c: np.ndarray, a_p: np.ndarray, i0: float):
    """Mean photon counts of both spectra for line integrals (a_c, a_p) (Eq. (2)).

    Returns (lam_high, lam_low); a plain sum over energy bins of the normalised
    spectrum times the Beer-Lambert transmission.
    """
    out = []
    for s in (spec.s_high, spec.s_low):
        w = s / s.sum()
        lam = np.zeros(a_c.shape)
        for k in np.nonzero(w)[0]:
            lam += w[k] * np.exp(-spec.f_kn[k] * a_c - spec.f_p[k] * a_p)
        out.append(i0 * lam)
    return out[0], out[1]


def poisson_counts(lam_high, lam_low, seed: int):
    """Poisson photon counts, one independent stream per spectrum."""
    rh = np.random.Generator(np.random.PCG64(np.random.SeedSequence([seed, 1])))
    rl = np.random.Generator(np.random.PCG64(np.random.SeedSequence([seed, 2])))
    return (rh.poisson(lam_high).astype(np.float64), rl.poisson(lam_low).astype(np.float64))


@dataclass
class Problem:
    """One reconstruction problem: geometry, spectra, photon counts and ground truth."""
    name: str
    geom: dict
    spec: Spectra
    i0: float
    counts_high: np.ndarray        # [V, D]
    counts_low: np.ndarray
    a_true: tuple                  # analytic (a_c, a_p), [V, D] each
    x_true: tuple | None           # (x_c, x_p), [ny, nx] each
    lam: float = 1e-5
    rho0: float = 1e-3
    iters: int = 50
    seed: int = 0


def make_problem(name: str, geom: dict, phantom: Phantom, i0: float, seed: int,
                 spec: Spectra | None = None, with_image: bool = True, noise: bool = True,
                 iters: int = 50) -> Problem:
    spec = default_spectra() if spec is None else spec
    ac, ap = phantom.line_integrals(geom)
    lh, ll = expected_counts(spec, ac, ap, i0)
    if noise:
        ch, cl = poisson_counts(lh, ll, seed)
    else:
        ch, cl = lh, ll
    xt = phantom.image(geom["nx"], geom["ny"], geom["pixel_cm"]) if with_image else None
    return Problem(name, geom, spec, i0, ch, cl, (ac, ap), xt, iters=iters, seed=seed)


def tiny_problem(seed: int = 0, **kw) -> Problem:
    """64x64 parallel beam, 90 views x 95 bins, 3 ellipses, I0 = 1e5, 20 iterations."""
    g = geometry("parallel", 64, 64, 0.5, 90, 95, 0.5)
    return make_problem("tiny64_parallel", g, tiny_phantom(seed), 1e5, seed, iters=20, **kw)


def slice_problem(seed: int = 0, n: int = 512, n_views: int = 720, n_det: int = 1024,
                  n_objects: int = 30, n_steel: int = 2, **kw) -> Problem:
    """Fan-beam luggage slice: 54/95 cm scanner, n^2 image over a 51.2 cm FOV, I0 = 2e5."""
    g = fan_geometry_fov(n, n_views, n_det)
    ph = luggage_phantom(seed, n_objects, n_steel)
    return make_problem(f"fan{n}_{n_views}x{n_det}", g, ph, 2e5, seed, **kw)


UNEVEN_CLASSES = ((256, 360, 512), (384, 540, 768), (512, 720, 1024))


def uneven_problem(index: int, base_seed: int = 1000, **kw) -> Problem:
    """Slice `index` of the uneven mix: sizes cycle 256/384/512, 10-40 objects, 0-3 steel."""
    n, V, D = UNEVEN_CLASSES[index % 3]
    seed = base_seed + index
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([seed, 7003])))
    n_obj = int(rng.integers(10, 41))
    n_steel = int(rng.integers(0, 4))
    return slice_problem(seed, n, V, D, n_obj, n_steel, **kw)
