"""Seeded synthetic light-field microscopy frames.

These stand in for the paper's bead, MCF-10A and zebrafish-vessel
acquisitions (Sec. 3), which are not available.  The recipe follows the
lenslet model of Sec. 2.1 / Fig. 1a: a frame is a grid of pitch x pitch
microlens images; an object point at lateral lens coordinates (X, Y) with a
depth slope k lights every lens (s, t) within 5 lenses with a Gaussian spot
whose in-lens centre shifts linearly with the lens offset.  Counts are
Poisson, plus a camera offset of 100 and Gaussian read noise of sigma 2,
rounded half-to-even and clipped to uint16.

This module holds no part of the compression method; both the GPU library's
tests and the oracle's tests draw their inputs from it.
"""
from __future__ import annotations

import numpy as np

PITCH = 15
OFFSET = 100.0
READ_SIGMA = 2.0
SPOT_SIGMA = 1.2
LENS_RADIUS = 5.0


def _add_spots(lam, X, Y, k, peak, pitch=PITCH, sigma=SPOT_SIGMA, radius=LENS_RADIUS):
    """Add one object point's light field into lam (float64, H x W)."""
    H, W = lam.shape
    ns, nt = H // pitch, W // pitch
    s0, s1 = max(0, int(np.floor(X - radius - 1))), min(ns, int(np.ceil(X + radius + 1)))
    t0, t1 = max(0, int(np.floor(Y - radius - 1))), min(nt, int(np.ceil(Y + radius + 1)))
    if s0 >= s1 or t0 >= t1:
        return
    s = np.arange(s0, s1)[:, None]
    t = np.arange(t0, t1)[None, :]
    ds = s + 0.5 - X
    dt = t + 0.5 - Y
    m = (ds * ds + dt * dt) <= radius * radius
    si, ti = np.nonzero(m)
    if si.size == 0:
        return
    ds_l = ds[si, 0]
    dt_l = dt[0, ti]
    c = (pitch - 1) / 2.0
    u0 = c + k * ds_l
    v0 = c + k * dt_l
    u = np.arange(pitch)[None, :]
    gu = np.exp(-((u - u0[:, None]) ** 2) / (2 * sigma * sigma))
    gv = np.exp(-((u - v0[:, None]) ** 2) / (2 * sigma * sigma))
    contrib = peak * gu[:, :, None] * gv[:, None, :]
    view = lam.reshape(ns, pitch, nt, pitch).transpose(0, 2, 1, 3)
    view[si + s0, ti + t0] += contrib


def _sensor(rng, lam):
    counts = rng.poisson(lam).astype(np.float64)
    noisy = counts + OFFSET + rng.normal(0.0, READ_SIGMA, size=lam.shape)
    return np.clip(np.rint(noisy), 0, 65535).astype(np.uint16)


def beads_frame(h=225, w=225, n_beads=20, peak=200.0, seed=1, pitch=PITCH, slope=0.5, depth_window=None,
                positions=None):
    """Bead light-field frame.  Draw order: bead parameters, Poisson, read noise.

    positions: optional (n, 3) array of (X, Y, k) to render instead of drawing.
    depth_window: optional (centre, half_width) for k instead of U[-slope, slope].
    Returns (frame uint16 [h, w], positions float64 [n, 3]).
    """
    rng = np.random.default_rng(seed)
    ns, nt = h // pitch, w // pitch
    if positions is None:
        X = rng.uniform(0, ns, n_beads)
        Y = rng.uniform(0, nt, n_beads)
        if depth_window is None:
            k = rng.uniform(-slope, slope, n_beads)
        else:
            k = rng.uniform(depth_window[0] - depth_window[1], depth_window[0] + depth_window[1], n_beads)
        positions = np.stack([X, Y, k], axis=1)
    lam = np.zeros((h, w), np.float64)
    for X, Y, k in positions:
        _add_spots(lam, X, Y, k, peak, pitch)
    return _sensor(rng, lam), positions


def config1_frame(seed=1):
    """225x225, 15x15 lenses, 20 beads, peak 200."""
    return beads_frame(225, 225, 20, 200.0, seed)[0]


def config2_frame(peak=100.0, seed=None):
    """2040x2040, 136x136 lenses, 2000 beads at peak 20 / 100 / 1000 (seeds 2 / 3 / 4)."""
    if seed is None:
        seed = {20.0: 2, 100.0: 3, 1000.0: 4}.get(float(peak), 3)
    return beads_frame(2040, 2040, 2000, float(peak), seed)[0]


# --------------------------------------------------------------------------- vessels
def _natural_cubic(ctrl, n_samples):
    """Natural cubic spline through control points (parameterised 0..len-1)."""
    from scipy.interpolate import CubicSpline

    tt = np.arange(len(ctrl))
    cs = CubicSpline(tt, ctrl, bc_type="natural")
    u = np.linspace(0, len(ctrl) - 1, n_samples)
    return cs(u)


class VesselScene:
    """Static tube light field plus particles advected along the tubes.

    Tubes: natural cubic splines through 4 seeded control points in lens
    units, radius U[3, 8] px, a depth slope per control point interpolated
    along the tube, about 300 photons added on axis over a background of
    300 photons.  Particles: peak 1000 photons, sigma 1.2 px, assigned to
    tubes and moved along arc length at U[2, 10] px per frame.
    """

    def __init__(self, seed=5, lenses=136, n_tubes=30, n_particles=500, pitch=PITCH, background=300.0,
                 tube_photons=300.0, particle_peak=1000.0):
        rng = np.random.default_rng(seed)
        self.pitch = pitch
        self.lenses = lenses
        H = W = lenses * pitch
        self.shape = (H, W)
        tubes = []
        for _ in range(n_tubes):
            ctrl = rng.uniform(0, lenses, size=(4, 2))
            kc = rng.uniform(-0.5, 0.5, size=4)
            radius = rng.uniform(3, 8)
            tubes.append((ctrl, kc, radius))
        parts = []
        for _ in range(n_particles):
            parts.append((int(rng.integers(0, n_tubes)), rng.uniform(0, 1), rng.uniform(2, 10)))
        self.seed = seed
        self.particle_peak = particle_peak
        # Static light field: point-sample each tube along its arc and across its
        # width; the summed tube field is then scaled so that its 99.9th
        # percentile adds `tube_photons` over the background.
        lam = np.zeros((H, W), np.float64)
        self.paths = []
        for ctrl, kc, radius in tubes:
            dense = _natural_cubic(np.concatenate([ctrl, kc[:, None]], axis=1), 2000)
            seg = np.sqrt(((dense[1:, :2] - dense[:-1, :2]) ** 2).sum(1))
            arc = np.concatenate([[0.0], np.cumsum(seg)])
            self.paths.append((dense, arc))
            step = 0.5  # lens units between samples along the arc
            n = max(2, int(arc[-1] / step))
            at = np.linspace(0, arc[-1], n)
            r_l = radius / pitch
            offs = np.linspace(-r_l, r_l, 3)
            for a in at:
                idx = min(len(arc) - 1, int(np.searchsorted(arc, a)))
                X, Y, k = dense[idx]
                if idx + 1 < len(dense):
                    d = dense[idx + 1, :2] - dense[idx, :2]
                else:
                    d = dense[idx, :2] - dense[idx - 1, :2]
                nrm = np.array([-d[1], d[0]]) / (np.hypot(d[0], d[1]) + 1e-12)
                for o in offs:
                    w = np.exp(-(o * o) / (2 * (r_l / 2 + 1e-9) ** 2))
                    _add_spots(lam, X + o * nrm[0], Y + o * nrm[1], k, w, pitch)
        lit = lam[lam > 0]
        scale = tube_photons / np.percentile(lit, 99.9) if lit.size else 0.0
        self.static = background + lam * scale
        self.particles = parts

    def frame(self, i, shape=None, rng=None):
        """Frame i of the series (optionally cropped top-left to shape)."""
        H, W = self.shape
        lam = self.static.copy()
        for tube, frac, speed in self.particles:
            dense, arc = self.paths[tube]
            a = (frac * arc[-1] + i * speed / self.pitch) % max(arc[-1], 1e-9)
            idx = min(len(arc) - 1, int(np.searchsorted(arc, a)))
            X, Y, k = dense[idx]
            _add_spots(lam, X, Y, k, self.particle_peak, self.pitch)
        if rng is None:
            rng = np.random.default_rng(self.seed * 100003 + i)
        if shape is not None:
            lam = lam[: shape[0], : shape[1]]
        return _sensor(rng, np.ascontiguousarray(lam))


SIZE_CLASSES = ((2040, 2040), (1020, 1020), (2040, 1020))


def vessel_series(n_frames=64, seed=5, lenses=136, sizes=SIZE_CLASSES):
    """Mixed-size time series: frame i has size class i mod 3 (top-left crops).

    Returns a list of (frame, prev_index or None); the temporal candidate of
    frame i refers to frame i-3, which has the same size class.
    """
    scene = VesselScene(seed=seed, lenses=lenses)
    frames = []
    for i in range(n_frames):
        shp = sizes[i % len(sizes)]
        shp = (min(shp[0], scene.shape[0]), min(shp[1], scene.shape[1]))
        frames.append(scene.frame(i, shp))
    return [(f, (i - len(sizes)) if i >= len(sizes) else None) for i, f in enumerate(frames)]


# --------------------------------------------------------------------------- adversarial content
def adversarial_frames(h=450, w=450, seed=9):
    """Frames that stress the codec's corner cases (names -> uint16 arrays)."""
    rng = np.random.default_rng(seed)
    out = {}
    out["zeros"] = np.zeros((h, w), np.uint16)
    out["const_0101"] = np.full((h, w), 0x0101, np.uint16)
    out["alt_0100"] = np.full((h, w), 0x0100, np.uint16)
    out["index"] = (np.arange(h * w, dtype=np.uint32) & 0xFFFF).astype(np.uint16).reshape(h, w)
    sat = np.full((h, w), 100, np.uint16)
    sat[h // 4: h // 2, w // 4: w // 2] = 65535
    out["saturated"] = sat
    out["uniform"] = rng.integers(0, 65536, size=(h, w), dtype=np.uint16)
    # bytes in groups "aaaa b": four equal bytes then another -> first-stage expansion 1.25
    pat = np.frombuffer(bytes([7, 7, 7, 7, 9] * ((2 * h * w) // 5 + 1)), np.uint8)[: 2 * h * w]
    out["four_run"] = pat.view(np.uint16).reshape(h, w).copy()
    out["period2"] = np.frombuffer(bytes([1, 2] * (h * w)), np.uint16).reshape(h, w).copy()
    p7 = np.frombuffer(bytes([3, 1, 4, 1, 5, 9, 2] * ((2 * h * w) // 7 + 1)), np.uint8)[: 2 * h * w]
    out["period7"] = p7.view(np.uint16).reshape(h, w).copy()
    return out


def long_tail_frame(h=450, w=450, seed=5, scale=16.0):
    """Bytes drawn independently with a geometric tail (byte v about
    2**(-v / scale) as likely as byte 0, 255 taking the rest): the rare bytes
    get Huffman codes longer than twelve bits."""
    rng = np.random.default_rng(seed)
    v = rng.geometric(1.0 - 2.0 ** (-1.0 / scale), size=2 * h * w) - 1
    return np.minimum(v, 255).astype(np.uint8).view(np.uint16).reshape(h, w).copy()
