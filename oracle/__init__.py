"""Plain FP64 CPU oracle of the splitting-based dual-energy CT ADMM.

TEST INFRASTRUCTURE ONLY: imported by the tests, by the smoke check and by the
benchmark's CPU-baseline leg, never by the reconstruction library.  It shares
no code with the GPU path; the two meet only in the seeded inputs.

The operators R, R^T, the forward transform f and the per-ray decomposition are
plain C (dect_oracle.c, double precision); everything else is numpy, written to
be read against the paper:

* Eq. (3)    forward transform f_s(a) = -ln sum_k w_s[k] exp(-f_KN[k] a_c - f_p[k] a_p)
* Eq. (4)    MAP objective 1/2 ||f(R x) - m||^2_Sigma + lambda |x|_TV + g(x)
* Eq. (9)    y = shrinkage(D x - u^y, lambda/rho)  (soft threshold)
* Eq. (10)   z = max(0, x - u^z)
* Eq. (11)   u <- u + [a; y; z] - [R; D; I] x
* Eq. (12)   x = argmin ||[a; y; z] - [R; D; I] x + [u^a; u^y; u^z]||^2, by CG, or by
             CG preconditioned with a high-pass (ramp) filter applied by 2-D FFT
             (Sec. 3.3: the system is shift-invariant once Sigma has moved to Eq. (13))
* Eq. (13)   a = argmin per ray 1/2 ||f(a) - m||^2_Sigma + sum_b rho_b/2 (a_b - R x_b + u^a_b)^2,
             by Levenberg-Marquardt
* Sec. 3.2   rho adapted from the primal and dual residuals (residual balancing)
* Eq. (14)   xi(x) = 20 log10(||x - x*|| / ||x*||)
* Table 1    operator counts per iteration: R 2n, R^T 2(n+1), f 4m
* Sec. 2     CDM: per-ray decomposition constrained to a >= 0 (projected LM with an active
             set), and FBP (Ram-Lak, parallel or flat-detector fan) of the line integrals
* Sec. 4     the initial image: x_c from CDM-FBP, x_p = x_c sum(a_p) / sum(a_c)
* Eqs. (7)-(8)  the baseline LM(m) x CG(n) splitting: x_c, then x_p, each by m LM
             iterations whose Gauss-Newton steps are n CG steps with R and R^T;
             Table 1: R 2m(n+1), R^T 2m(n+1), f 4m

Readings where the paper is silent (each listed with its reason in the design
notes): the ramp preconditioner is max(|w|, 1/P) in cycles per pixel on a
zero-padded grid of P = powers of two at least twice each image side (a pure
ramp vanishes at w = 0); Sigma = diag(counts / I0); anisotropic TV with forward differences and a
zero last difference; LM damping mu0 = 1e-3 reset every outer iteration, x10 / /10,
Marquardt scaling; residual balancing with mu = 10 and tau = 2; initial state
x = 0 and a from a rho = 0 decomposition started at the linearised solution.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass, field

import numpy as np

from . import build as _build

_LIB = None


def _lib():
    global _LIB
    if _LIB is None:
        path = _build.LIB
        if not os.path.exists(path) or os.path.getmtime(path) < os.path.getmtime(_build.SRC):
            _build.build()
        _LIB = ctypes.CDLL(path)
        P = ctypes.POINTER
        d, i, l = ctypes.c_double, ctypes.c_int, ctypes.c_long
        pd = P(d)
        _LIB.orc_project.argtypes = [P(_Geom), pd, pd]
        _LIB.orc_backproject.argtypes = [P(_Geom), pd, pd]
        _LIB.orc_forward.argtypes = [i, pd, pd, pd, i, pd, pd, pd, l, pd, pd, pd, pd, pd, pd]
        _LIB.orc_udm.argtypes = [i, pd, pd, pd, i, pd, pd, pd, l, pd, pd, pd, pd, pd, pd, d, d, i,
                                 d, pd, pd, pd, P(ctypes.c_uint8), pd]
        _LIB.orc_udm.restype = i
        _LIB.orc_cdm.argtypes = [i, pd, pd, pd, i, pd, pd, pd, l, pd, pd, pd, pd, i, d, pd, pd, pd]
        _LIB.orc_cdm.restype = i
        _LIB.orc_set_threads.argtypes = [i]
        _LIB.orc_max_threads.restype = i
    return _LIB


def set_threads(n: int) -> None:
    """Threads of the C part's parallel loops (results do not depend on it)."""
    _lib().orc_set_threads(int(n))


def max_threads() -> int:
    return int(_lib().orc_max_threads())


class _Geom(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int), ("nx", ctypes.c_int), ("ny", ctypes.c_int),
                ("pixel", ctypes.c_double), ("n_views", ctypes.c_int), ("n_det", ctypes.c_int),
                ("det_cm", ctypes.c_double), ("det_offset", ctypes.c_double),
                ("src_iso", ctypes.c_double), ("src_det", ctypes.c_double),
                ("angle0", ctypes.c_double), ("span", ctypes.c_double)]


def _ptr(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double)) if a is not None else None


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


# -----------------------------------------------------------------------------
# Finite differences (Eq. (5)): forward differences, last difference zero.
# -----------------------------------------------------------------------------

def D(x: np.ndarray) -> np.ndarray:
    """[2, ny, nx]: horizontal then vertical forward differences of x [ny, nx]."""
    out = np.zeros((2,) + x.shape)
    out[0, :, :-1] = x[:, 1:] - x[:, :-1]
    out[1, :-1, :] = x[1:, :] - x[:-1, :]
    return out


def DT(y: np.ndarray) -> np.ndarray:
    """Transpose of D."""
    h, v = y[0], y[1]
    out = np.zeros(h.shape)
    out[:, :-1] -= h[:, :-1]
    out[:, 1:] += h[:, :-1]
    out[:-1, :] -= v[:-1, :]
    out[1:, :] += v[:-1, :]
    return out


def pad_shape(ny: int, nx: int) -> tuple:
    """Padded FFT grid: the smallest powers of two at least twice each image side, so
    that the filter acts as a linear (not circular) convolution over the image."""
    def up(n):
        p = 1
        while p < 2 * n:
            p *= 2
        return p
    return up(ny), up(nx)


def ramp_filter(py: int, px: int) -> np.ndarray:
    """Floored ramp max(|w|, 1/max(py, px)) on the py x px DFT grid, |w| in cycles per
    pixel (the ramp filter as the CG preconditioner, Sec. 3.3)."""
    fy = np.fft.fftfreq(py)[:, None]
    fx = np.fft.fftfreq(px)[None, :]
    return np.maximum(np.sqrt(fy * fy + fx * fx), 1.0 / max(py, px))


def precondition(img: np.ndarray, filt: np.ndarray) -> np.ndarray:
    """M r: zero-pad the image to the filter's grid, multiply its 2-D DFT by the
    filter, transform back and keep the image's own pixels."""
    ny, nx = img.shape
    pad = np.zeros(filt.shape)
    pad[:ny, :nx] = img
    return np.real(np.fft.ifft2(np.fft.fft2(pad) * filt))[:ny, :nx]


def ramlak_kernel(P: int, delta: float) -> np.ndarray:
    """Discrete ramp (Ram-Lak) kernel of sample spacing delta, circularly indexed over
    P samples: h[0] = 1/(4 delta^2), h[n] = -1/(pi^2 n^2 delta^2) for odd n, 0 for
    even n != 0 (the band-limited ramp sampled at n delta)."""
    h = np.zeros(P)
    n = np.arange(P)
    n = np.where(n < P // 2, n, n - P)
    odd = (n % 2) != 0
    h[odd] = -1.0 / (np.pi ** 2 * n[odd].astype(float) ** 2 * delta ** 2)
    h[0] = 1.0 / (4.0 * delta ** 2)
    return h


def shrink(v: np.ndarray, t: float) -> np.ndarray:
    """Soft threshold: the minimiser of t|y| + 1/2 (y - v)^2 (Eq. (9))."""
    return np.sign(v) * np.maximum(np.abs(v) - t, 0.0)


def xi_db(x: np.ndarray, x_true: np.ndarray) -> float:
    """Eq. (14): normalised l2 distance to the ground truth, in dB."""
    return 20.0 * np.log10(np.linalg.norm(x - x_true) / np.linalg.norm(x_true))


def ingest(counts: np.ndarray, i0: float):
    """Log measurement m = ln(I0 / max(c, 1)) and weight w = c / I0 (Sigma = diag(counts))."""
    c = np.asarray(counts, dtype=np.float64)
    return np.log(i0 / np.maximum(c, 1.0)), c / i0


# -----------------------------------------------------------------------------
# State and parameters
# -----------------------------------------------------------------------------


@dataclass
class Params:
    lam: tuple = (1e-5, 1e-5)        # lambda_c, lambda_p (Sec. 4)
    rho0: tuple = (1e-3, 1e-3)       # initial rho_c, rho_p (Sec. 4)
    lm_iters: int = 1                # m
    cg_iters: int = 1                # n
    rho_mode: str = "adaptive"       # "adaptive" | "fixed"
    bal_mu: float = 10.0
    bal_tau: float = 2.0
    lm_mu0: float = 1e-3
    precond: str | None = None       # None (CG) or "ramp" (PCG)


@dataclass
class State:
    """Full ADMM state, per basis b in (c, p): index 0 = Compton, 1 = photoelectric."""
    x: np.ndarray      # [2, ny, nx]
    Rx: np.ndarray     # [2, V, D], tracked R x
    a: np.ndarray      # [2, V, D]
    ua: np.ndarray     # [2, V, D]
    y: np.ndarray      # [2, 2, ny, nx]
    uy: np.ndarray     # [2, 2, ny, nx]
    z: np.ndarray      # [2, ny, nx]
    uz: np.ndarray     # [2, ny, nx]
    rho: np.ndarray    # [2]
    it: int = 0
    log: list = field(default_factory=list)
    lm_ties: np.ndarray | None = None  # per-ray near-tie ratios of the last replayed a-update

    def copy(self):
        return State(*(np.array(getattr(self, k)) for k in
                       ("x", "Rx", "a", "ua", "y", "uy", "z", "uz", "rho")),
                     it=self.it, log=list(self.log))


class Oracle:
    """FP64 reference for one geometry and one pair of spectra."""

    def __init__(self, geom: dict, spec):
        self.geom = dict(geom)
        g = _Geom()
        g.kind = 0 if geom["kind"] == "parallel" else 1
        for k in ("nx", "ny", "n_views", "n_det"):
            setattr(g, k, int(geom[k]))
        g.pixel = geom["pixel_cm"]
        g.det_cm = geom["det_cm"]
        g.det_offset = geom["det_offset"]
        g.src_iso = geom["src_iso_cm"]
        g.src_det = geom["src_det_cm"]
        g.angle0 = geom["angle0"]
        g.span = geom["span"]
        self._g = g
        self.img_shape = (int(geom["ny"]), int(geom["nx"]))
        self.sino_shape = (int(geom["n_views"]), int(geom["n_det"]))
        # Normalised spectra restricted to their nonzero bins (the constant C_s of
        # Eq. (3) makes f independent of the scale of S).
        self._spec = []
        self.mean_f = []
        for s in (spec.s_high, spec.s_low):
            s = np.asarray(s, dtype=np.float64)
            nz = np.nonzero(s > 0)[0]
            w = s[nz] / s.sum()
            fkn = _f64(np.asarray(spec.f_kn)[nz])
            fp = _f64(np.asarray(spec.f_p)[nz])
            self._spec.append((len(nz), _f64(np.log(w)), fkn, fp))
            self.mean_f.append((float(np.sum(w * fkn)), float(np.sum(w * fp))))
        self.counts = {"R": 0, "RT": 0, "RT_dual": 0, "f": 0}

    # -- tomographic operators ------------------------------------------------
    def project(self, img: np.ndarray, count: str | None = "R") -> np.ndarray:
        img = _f64(img)
        assert img.shape == self.img_shape
        out = np.empty(self.sino_shape)
        _lib().orc_project(ctypes.byref(self._g), _ptr(img), _ptr(out))
        if count:
            self.counts[count] += 1
        return out

    def backproject(self, sino: np.ndarray, count: str = "RT") -> np.ndarray:
        sino = _f64(sino)
        assert sino.shape == self.sino_shape
        out = np.empty(self.img_shape)
        _lib().orc_backproject(ctypes.byref(self._g), _ptr(sino), _ptr(out))
        self.counts[count] += 1
        return out

    # -- forward transform and decomposition -----------------------------------
    def _spec_args(self):
        (nh, lh, kh, ph), (nl, ll, kl, pl) = self._spec
        return [nh, _ptr(lh), _ptr(kh), _ptr(ph), nl, _ptr(ll), _ptr(kl), _ptr(pl)]

    def forward(self, a_c, a_p):
        """f_h, f_l and their gradients [.., 2] at line integrals (a_c, a_p) (Eq. (3))."""
        ac, ap = _f64(a_c), _f64(a_p)
        n = ac.size
        fh, fl = np.empty(n), np.empty(n)
        gh, gl = np.empty(2 * n), np.empty(2 * n)
        _lib().orc_forward(*self._spec_args(), n, _ptr(ac), _ptr(ap), _ptr(fh), _ptr(fl),
                           _ptr(gh), _ptr(gl))
        sh = ac.shape
        return fh.reshape(sh), fl.reshape(sh), gh.reshape(sh + (2,)), gl.reshape(sh + (2,))

    def udm(self, mh, ml, wh, wl, vc, vp, rho_c, rho_p, iters, a_c, a_p, mu0=1e-3,
            force=None, ties: list | None = None):
        """Eq. (13) per ray by `iters` LM iterations from (a_c, a_p); returns (a_c, a_p, Phi).

        force: optional uint8 array of the rays' shape whose bit k replays the accept
        decision of LM iteration k (k < 8) taken elsewhere, e.g. by single-precision
        arithmetic.  The per-ray near-tie ratios of replayed decisions that disagree with
        this one's own comparison (|Phi(trial) - Phi(current)| over their single-precision
        rounding scale; 0 where none disagrees) are appended to `ties` if given."""
        sh = np.shape(a_c)
        ac, ap = _f64(a_c).ravel().copy(), _f64(a_p).ravel().copy()
        n = ac.size
        args = [_f64(v).ravel() if v is not None else None for v in (mh, ml, wh, wl, vc, vp)]
        phi = np.empty(n)
        fz = None
        tie = None
        if force is not None:
            fz = np.ascontiguousarray(force, dtype=np.uint8).ravel()
            assert fz.size == n
            tie = np.empty(n)
        nf = _lib().orc_udm(*self._spec_args(), n, *(_ptr(v) for v in args), float(rho_c),
                            float(rho_p), int(iters), float(mu0), _ptr(ac), _ptr(ap), _ptr(phi),
                            fz.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)) if fz is not None
                            else None, _ptr(tie))
        self.counts["f"] += nf
        if ties is not None and tie is not None:
            ties.append(tie.reshape(sh))
        return ac.reshape(sh), ap.reshape(sh), phi.reshape(sh)

    def cdm(self, mh, ml, wh, wl, iters=20, mu0=1e-3):
        """Constrained decomposition (CDM): per ray, 1/2 ||f(a) - m||^2_Sigma over a >= 0 by
        projected LM from the linearised solution (projected); returns (a_c, a_p)."""
        c0, p0 = self.linearised(mh, ml)
        sh = np.shape(mh)
        ac, ap = _f64(c0).ravel().copy(), _f64(p0).ravel().copy()
        n = ac.size
        args = [_f64(v).ravel() for v in (mh, ml, wh, wl)]
        nf = _lib().orc_cdm(*self._spec_args(), n, *(_ptr(v) for v in args), int(iters),
                            float(mu0), _ptr(ac), _ptr(ap), None)
        self.counts["f"] += nf
        return ac.reshape(sh), ap.reshape(sh)

    def fbp(self, sino: np.ndarray) -> np.ndarray:
        """Filtered backprojection of line integrals [V, D] (Kak and Slaney): parallel beam
        x = (span/V) sum_v q_v(s), q_v = delta (p_v * h); equispaced fan beam with the
        detector scaled to the isocentre (spacing delta), x = (span/V) sum_v U^-2 q_v(s),
        q_v = delta (R'_v * h) / 2, R' = R D / sqrt(D^2 + s^2), U = L / D; h the Ram-Lak
        kernel, linear interpolation in s, zero outside the detector."""
        g = self.geom
        V, Dn = self.sino_shape
        ny, nx = self.img_shape
        P = 1
        while P < 2 * Dn:
            P *= 2
        fan = g["kind"] == "fan"
        delta = g["det_cm"] * (g["src_iso_cm"] / g["src_det_cm"] if fan else 1.0)
        u = (np.arange(Dn) - 0.5 * (Dn - 1) + g["det_offset"]) * delta
        pre = np.asarray(sino, dtype=np.float64)
        if fan:
            Dsrc = g["src_iso_cm"]
            pre = pre * (Dsrc / np.sqrt(Dsrc ** 2 + u ** 2))[None, :]
        H = np.fft.fft(ramlak_kernel(P, delta))
        pad = np.zeros((V, P))
        pad[:, :Dn] = pre
        q = delta * np.real(np.fft.ifft(np.fft.fft(pad, axis=1) * H[None, :], axis=1))[:, :Dn]
        if fan:
            q *= 0.5
        xs = (np.arange(nx) - 0.5 * (nx - 1)) * g["pixel_cm"]
        ys = (np.arange(ny) - 0.5 * (ny - 1)) * g["pixel_cm"]
        X, Y = np.meshgrid(xs, ys)
        img = np.zeros((ny, nx))
        for v in range(V):
            t = g["angle0"] + v * g["span"] / V
            c, sn = np.cos(t), np.sin(t)
            if fan:
                L = g["src_iso_cm"] - (X * c + Y * sn)
                s_iso = g["src_iso_cm"] * (-X * sn + Y * c) / L
                w = (g["src_iso_cm"] / L) ** 2
            else:
                s_iso = X * c + Y * sn
                w = 1.0
            b = s_iso / delta + 0.5 * (Dn - 1) - g["det_offset"]
            b0 = np.floor(b)
            al = b - b0
            i0 = b0.astype(np.int64)
            v0 = np.where((i0 >= 0) & (i0 < Dn), q[v, np.clip(i0, 0, Dn - 1)], 0.0)
            v1 = np.where((i0 + 1 >= 0) & (i0 + 1 < Dn), q[v, np.clip(i0 + 1, 0, Dn - 1)], 0.0)
            img += w * ((1.0 - al) * v0 + al * v1)
        return img * (g["span"] / V)

    def cdm_fbp(self, mh, ml, wh, wl, iters=20):
        """The projection-wise baseline: CDM line integrals, then FBP of each basis."""
        ac, ap = self.cdm(mh, ml, wh, wl, iters)
        return (ac, ap), np.stack([self.fbp(ac), self.fbp(ap)])

    def linearised(self, mh, ml):
        """a solving the 2x2 linearisation of f at a = 0 (rows = spectrum-mean f_KN, f_p)."""
        (hc, hp), (lc, lp) = self.mean_f
        det = hc * lp - hp * lc
        return (lp * mh - hp * ml) / det, (hc * ml - lc * mh) / det

    # -- objectives ------------------------------------------------------------
    def data_cost(self, a_c, a_p, mh, ml, wh, wl) -> float:
        fh, fl, _, _ = self.forward(a_c, a_p)
        return 0.5 * float(np.sum(wh * (fh - mh) ** 2) + np.sum(wl * (fl - ml) ** 2))

    def map_objective(self, x, mh, ml, wh, wl, lam) -> float:
        """Eq. (4) at the nonnegative part of x (where g = 0)."""
        xp = np.maximum(x, 0.0)
        a = [self.project(xp[b], count=None) for b in range(2)]
        tv = sum(lam[b] * np.abs(D(xp[b])).sum() for b in range(2))
        return self.data_cost(a[0], a[1], mh, ml, wh, wl) + tv

    def split_objective(self, st: State, mh, ml, wh, wl, lam) -> float:
        return (self.data_cost(st.a[0], st.a[1], mh, ml, wh, wl)
                + sum(lam[b] * np.abs(st.y[b]).sum() for b in range(2)))

    # -- ADMM ------------------------------------------------------------------
    def admm_init(self, mh, ml, wh, wl, params: Params, init_iters: int = 10,
                  x0: np.ndarray | None = None) -> State:
        """a from a rho = 0 decomposition started at the linearised solution; x = 0, or
        x = x0 [2, ny, nx] with R x = R x0, y = D x0, z = x0 and u = 0."""
        ny, nx = self.img_shape
        V, Dn = self.sino_shape
        ac, ap = self.linearised(mh, ml)
        ac, ap, _ = self.udm(mh, ml, wh, wl, None, None, 0.0, 0.0, init_iters, ac, ap,
                             params.lm_mu0)
        z2 = lambda *s: np.zeros((2,) + s)
        st = State(x=z2(ny, nx), Rx=z2(V, Dn), a=np.stack([ac, ap]), ua=z2(V, Dn),
                   y=z2(2, ny, nx), uy=z2(2, ny, nx), z=z2(ny, nx), uz=z2(ny, nx),
                   rho=np.array(params.rho0, dtype=np.float64))
        if x0 is not None:
            st.x = np.array(x0, dtype=np.float64)
            st.z = st.x.copy()
            for b in range(2):
                st.Rx[b] = self.project(st.x[b], count=None)
                st.y[b] = D(st.x[b])
        return st

    def cdm_fbp_start(self, mh, ml, wh, wl, cdm_iters=20) -> np.ndarray:
        """The paper's initial image (Sec. 4): the CDM-FBP Compton image, and for the
        photoelectric image that Compton image scaled by sum(a_p) / sum(a_c) over the
        CDM line integrals."""
        (ac, ap), x = self.cdm_fbp(mh, ml, wh, wl, cdm_iters)
        return np.stack([x[0], (float(np.sum(ap)) / float(np.sum(ac))) * x[0]])

    def cg(self, x, Rx, rhs_sino, rhs_img, n, filt=None):
        """n CG iterations on (R^T R + D^T D + I) x = R^T rhs_sino + rhs_img (Eq. (12)),
        warm-started at x with R x = Rx known; returns (x, Rx) with Rx kept equal to R x.
        With a filter, preconditioned CG with M = precondition(., filt)."""
        M = (lambda v: v) if filt is None else (lambda v: precondition(v, filt))
        r = self.backproject(rhs_sino - Rx) + rhs_img - DT(D(x)) - x
        zv = M(r)
        p = zv.copy()
        gamma = float(np.dot(r.ravel(), zv.ravel()))
        for _ in range(n):
            if gamma == 0.0:
                break
            Rp = self.project(p)
            q = self.backproject(Rp) + DT(D(p)) + p
            alpha = gamma / float(np.dot(p.ravel(), q.ravel()))
            x = x + alpha * p
            Rx = Rx + alpha * Rp
            r = r - alpha * q
            zv = M(r)
            gamma_new = float(np.dot(r.ravel(), zv.ravel()))
            p = zv + (gamma_new / gamma) * p
            gamma = gamma_new
        return x, Rx

    def admm_iterate(self, st: State, mh, ml, wh, wl, params: Params, n_iters: int = 1,
                     lm_force=None, rho_force=None) -> State:
        """n_iters ADMM iterations: x (Eq. 12), a (Eq. 13), y and z (Eq. 9-10), u (Eq. 11), rho.

        Replays for parity runs against single-precision arithmetic, whose discrete
        decisions can differ from this one's on near-ties: lm_force[k] (uint8 [V, D], see
        udm) replays the LM accept decisions of iteration k, and the log records how close
        every replayed decision that differs from this one's own was ('lm_tie_max', 0 if
        none; 'lm_flips', their count); rho_force[k] = (rho_c, rho_p) replaces the
        residual-balancing rho chosen at the end of iteration k, and 'rho_tie' records how
        far from a tie of the balancing test any differing decision of this one's was
        (|max(r, s) - mu min(r, s)| / max(r, s); 0 if none differs)."""
        st = st.copy()
        filt = None
        if params.precond == "ramp":
            filt = ramp_filter(*pad_shape(*self.img_shape))
        elif params.precond is not None:
            raise ValueError(f"unknown preconditioner {params.precond!r}")
        for it_k in range(n_iters):
            rho = st.rho.copy()
            a_prev, y_prev, z_prev = st.a.copy(), st.y.copy(), st.z.copy()
            # x-update, independently per basis (Eq. (12)); rho cancels.
            for b in range(2):
                st.x[b], st.Rx[b] = self.cg(
                    st.x[b], st.Rx[b], st.a[b] + st.ua[b],
                    DT(st.y[b] + st.uy[b]) + st.z[b] + st.uz[b], params.cg_iters, filt)
            # a-update: per-ray decomposition (Eq. (13)) with v = R x - u^a.
            v = st.Rx - st.ua
            ties = []
            force = lm_force[it_k] if lm_force is not None else None
            ac, ap, _ = self.udm(mh, ml, wh, wl, v[0], v[1], rho[0], rho[1], params.lm_iters,
                                 st.a[0], st.a[1], params.lm_mu0, force=force, ties=ties)
            st.a = np.stack([ac, ap])
            # y and z updates (Eq. (9)-(10)) and the scaled duals (Eq. (11)).
            for b in range(2):
                Dx = D(st.x[b])
                st.y[b] = shrink(Dx - st.uy[b], params.lam[b] / rho[b])
                st.z[b] = np.maximum(0.0, st.x[b] - st.uz[b])
                st.ua[b] += st.a[b] - st.Rx[b]
                st.uy[b] += st.y[b] - Dx
                st.uz[b] += st.z[b] - st.x[b]
            # Residuals and the rho update (residual balancing).
            r_norm = np.zeros(2)
            s_norm = np.zeros(2)
            for b in range(2):
                r_norm[b] = np.sqrt(np.sum((st.a[b] - st.Rx[b]) ** 2)
                                    + np.sum((st.y[b] - D(st.x[b])) ** 2)
                                    + np.sum((st.z[b] - st.x[b]) ** 2))
                if params.rho_mode == "adaptive":
                    sv = (self.backproject(st.a[b] - a_prev[b], count="RT_dual")
                          + DT(st.y[b] - y_prev[b]) + (st.z[b] - z_prev[b]))
                    s_norm[b] = rho[b] * np.linalg.norm(sv)
            new_rho = rho.copy()
            if params.rho_mode == "adaptive":
                for b in range(2):
                    if r_norm[b] > params.bal_mu * s_norm[b]:
                        new_rho[b] = rho[b] * params.bal_tau
                    elif s_norm[b] > params.bal_mu * r_norm[b]:
                        new_rho[b] = rho[b] / params.bal_tau
            rho_tie = 0.0
            if rho_force is not None:
                forced = np.array(rho_force[it_k], dtype=np.float64)
                for b in range(2):
                    if forced[b] != new_rho[b]:
                        # How close the balancing test r > mu s (or s > mu r) was to a tie.
                        hi, lo = max(r_norm[b], s_norm[b]), min(r_norm[b], s_norm[b])
                        rho_tie = max(rho_tie, abs(hi - params.bal_mu * lo) / max(hi, 1e-300))
                new_rho = forced
            for b in range(2):
                k = rho[b] / new_rho[b]
                st.ua[b] *= k
                st.uy[b] *= k
                st.uz[b] *= k
            st.rho = new_rho
            # The split objective's two terms: the data fit at the new a (Eq. (13)'s first
            # term) and lambda |y|_1 at the new y (Eq. (9)).
            data = self.data_cost(st.a[0], st.a[1], mh, ml, wh, wl)
            tv = sum(params.lam[b] * float(np.abs(st.y[b]).sum()) for b in range(2))
            entry = dict(it=st.it, rho=rho.copy(), r=r_norm.copy(), s=s_norm.copy(),
                         data=data, tv=tv, phi=data + tv)
            if ties:
                entry["lm_flips"] = int(np.count_nonzero(ties[0]))
                entry["lm_tie_max"] = float(ties[0].max())
                st.lm_ties = ties[0]
            if rho_force is not None:
                entry["rho_tie"] = rho_tie
            st.log.append(entry)
            st.it += 1
        return st

    # -- LM(m) x CG(n): the baseline splitting of Eqs. (7)-(8) -------------------
    def lmcg_init(self, mh, ml, wh, wl, params: Params, x0: np.ndarray | None = None):
        """x = x0 [2, ny, nx] (or 0), y = D x, z = x, u = 0, R x, and f, grad f at R x."""
        ny, nx = self.img_shape
        x = np.zeros((2, ny, nx)) if x0 is None else np.array(x0, dtype=np.float64)
        Rx = np.stack([self.project(x[b], count=None) for b in range(2)])
        fh, fl, gh, gl = self.forward(Rx[0], Rx[1])
        return LmcgState(x=x, Rx=Rx, y=np.stack([D(x[b]) for b in range(2)]),
                         uy=np.zeros((2, 2, ny, nx)), z=x.copy(), uz=np.zeros((2, ny, nx)),
                         rho=np.array(params.rho0, dtype=np.float64), fh=fh, fl=fl, gh=gh, gl=gl)

    def _lm_basis(self, st: LmcgState, b: int, mh, ml, wh, wl, rho: float, params: Params):
        """Eq. (7) (b = 0) or Eq. (8) (b = 1): m LM iterations on
        Phi(x_b) = 1/2 ||f(R x_c, R x_p) - m||^2_Sigma + rho/2 ||[y_b; z_b] - [D; I] x_b + u_b||^2
        with the other basis fixed.  Gauss-Newton curvature H = R^T W R + rho (D^T D + I),
        W = sum_s w_s (df_s/da_b)^2 per ray; the damped system (H + mu kappa I) d = -grad Phi,
        kappa = g^T H g / g^T g (the curvature along the gradient, from the first CG step),
        is solved by n CG steps from d = 0; the step is accepted if Phi decreases
        (mu / 10), else rejected (mu * 10); mu starts at lm_mu0 for every basis update."""
        y, uy, z, uz = st.y[b], st.uy[b], st.z[b], st.uz[b]

        def pen(x):
            return 0.5 * rho * (float(np.sum((y - D(x) + uy) ** 2)) + float(np.sum((z - x + uz) ** 2)))

        def data(fh, fl):
            return 0.5 * float(np.sum(wh * (fh - mh) ** 2) + np.sum(wl * (fl - ml) ** 2))

        mu = params.lm_mu0
        for _ in range(params.lm_iters):
            x = st.x[b]
            Jh, Jl = st.gh[..., b], st.gl[..., b]
            eh, el = st.fh - mh, st.fl - ml
            t = wh * eh * Jh + wl * el * Jl
            W = wh * Jh ** 2 + wl * Jl ** 2
            phi = data(st.fh, st.fl) + pen(x)
            g = self.backproject(t) + rho * (DT(D(x)) + x - DT(y + uy) - z - uz)

            def H(v):
                return self.backproject(W * self.project(v)) + rho * (DT(D(v)) + v)

            d = np.zeros_like(x)
            r = -g
            p = r.copy()
            rr = float(np.sum(r * r))
            kappa = None
            for _ in range(params.cg_iters):
                Hp = H(p)
                pp = float(np.sum(p * p))
                if kappa is None:
                    kappa = float(np.sum(p * Hp)) / pp if pp > 0 else 0.0
                q = Hp + mu * kappa * p
                pq = float(np.sum(p * q))
                alpha = rr / pq if pq > 0 else 0.0
                d = d + alpha * p
                r = r - alpha * q
                rr_new = float(np.sum(r * r))
                p = r + (rr_new / rr if rr > 0 else 0.0) * p
                rr = rr_new
            xt = x + d
            at = self.project(xt)
            pair = (at, st.Rx[1]) if b == 0 else (st.Rx[0], at)
            fh, fl, gh, gl = self.forward(*pair)
            self.counts["f"] += 2  # both spectra, every ray
            if data(fh, fl) + pen(xt) < phi:
                st.x[b], st.Rx[b] = xt, at
                st.fh, st.fl, st.gh, st.gl = fh, fl, gh, gl
                mu /= 10.0
            else:
                mu *= 10.0
        return st

    def lmcg_iterate(self, st: LmcgState, mh, ml, wh, wl, params: Params,
                     n_iters: int = 1) -> LmcgState:
        """n_iters outer iterations: x_c (Eq. 7), then x_p with the new x_c (Eq. 8), y and z
        (Eq. 9-10), u (Eq. 11 with C = [D; I]), then rho from the residuals."""
        st = st.copy()
        for _ in range(n_iters):
            rho = st.rho.copy()
            y_prev, z_prev = st.y.copy(), st.z.copy()
            for b in range(2):
                st = self._lm_basis(st, b, mh, ml, wh, wl, rho[b], params)
            r_norm, s_norm = np.zeros(2), np.zeros(2)
            for b in range(2):
                Dx = D(st.x[b])
                st.y[b] = shrink(Dx - st.uy[b], params.lam[b] / rho[b])
                st.z[b] = np.maximum(0.0, st.x[b] - st.uz[b])
                st.uy[b] += st.y[b] - Dx
                st.uz[b] += st.z[b] - st.x[b]
                r_norm[b] = np.sqrt(np.sum((st.y[b] - Dx) ** 2) + np.sum((st.z[b] - st.x[b]) ** 2))
                if params.rho_mode == "adaptive":
                    s_norm[b] = rho[b] * np.linalg.norm(DT(st.y[b] - y_prev[b]) + st.z[b] - z_prev[b])
            new_rho = rho.copy()
            if params.rho_mode == "adaptive":
                for b in range(2):
                    if r_norm[b] > params.bal_mu * s_norm[b]:
                        new_rho[b] = rho[b] * params.bal_tau
                    elif s_norm[b] > params.bal_mu * r_norm[b]:
                        new_rho[b] = rho[b] / params.bal_tau
            for b in range(2):
                k = rho[b] / new_rho[b]
                st.uy[b] *= k
                st.uz[b] *= k
            st.rho = new_rho
            data = 0.5 * float(np.sum(wh * (st.fh - mh) ** 2) + np.sum(wl * (st.fl - ml) ** 2))
            tv = sum(params.lam[b] * float(np.abs(st.y[b]).sum()) for b in range(2))
            st.log.append(dict(it=st.it, rho=rho.copy(), r=r_norm.copy(), s=s_norm.copy(),
                               data=data, tv=tv))
            st.it += 1
        return st


@dataclass
class LmcgState:
    """State of the LM x CG scheme, per basis b: x, R x (the projection of the accepted x),
    y, u^y, z, u^z, rho; f_h, f_l and their gradients [.., (c, p)] at R x."""
    x: np.ndarray      # [2, ny, nx]
    Rx: np.ndarray     # [2, V, D]
    y: np.ndarray      # [2, 2, ny, nx]
    uy: np.ndarray     # [2, 2, ny, nx]
    z: np.ndarray      # [2, ny, nx]
    uz: np.ndarray     # [2, ny, nx]
    rho: np.ndarray    # [2]
    fh: np.ndarray     # [V, D]
    fl: np.ndarray     # [V, D]
    gh: np.ndarray     # [V, D, 2]
    gl: np.ndarray     # [V, D, 2]
    it: int = 0
    log: list = field(default_factory=list)

    def copy(self):
        return LmcgState(*(np.array(getattr(self, k)) for k in
                           ("x", "Rx", "y", "uy", "z", "uz", "rho", "fh", "fl", "gh", "gl")),
                         it=self.it, log=list(self.log))
