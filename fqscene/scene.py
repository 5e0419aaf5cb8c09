"""Seeded scatterer scenes: static or moving tissue plus Poiseuille blood.

Scatterers follow the paper's model of tissue microstructure as random point
scatterers with reflection coefficients (Section 2.2.1), tissue and blood are
kept as separate sets (Section 2.3, Algorithm 1), and every trajectory is a
closed-form solution of the trajectory integral of Section 2.2.2 for a
steady field:
  * tissue (and the vessels embedded in it): rigid translation d(t);
    'static' gives d = 0, 'cardiac_resp' gives
    d(t) = 100 um sin(2 pi 1 Hz t) z + 300 um sin(2 pi 0.25 Hz t) (x + z)/sqrt(2);
  * blood: laminar Poiseuille flow along each vessel axis,
    v(r) = vmax (1 - r^2 / R^2), with periodic re-entry along the segment.
Frame f is sampled at t_f = f / PRF; the transmits of one frame see the
same positions.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional

import numpy as np

from .configs import Config


@dataclasses.dataclass
class Vessel:
    centre: np.ndarray      # (3,) m, at t = 0
    axis: np.ndarray        # (3,) unit vector, flow direction
    radius: float           # m
    half_len: float         # m
    vmax: float             # m/s (centre-line speed)


@dataclasses.dataclass
class Scene:
    tissue_pos: np.ndarray   # float32 [Ft][St][3]; Ft == 1 when the tissue is static
    tissue_amp: np.ndarray   # float32 [St]
    blood_pos: np.ndarray    # float32 [F][Sb][3]
    blood_amp: np.ndarray    # float32 [Sb]
    vessels: List[Vessel]
    blood_vessel: np.ndarray  # int32 [Sb] vessel index of each blood scatterer
    blood_radial: np.ndarray  # float64 [Sb] radial distance / R
    times: np.ndarray         # float64 [F] frame times, s

    @property
    def tissue_static(self) -> bool:
        return self.tissue_pos.shape[0] == 1


def rigid_motion(spec, t: np.ndarray):
    """Closed-form solution of the trajectory integral (Section 2.2.2) for the tissue
    velocity fields: p(t) = c + R(t) (p0 - c) + d(t).  Returns R [F][3][3], d [F][3],
    c [3].  'velocity': d = V t.  'rotation': V(r) = W x (r - c) with W = (0, -w, 0), whose
    solution rotates about the -y axis through c by the angle w t."""
    t = np.asarray(t, dtype=np.float64)
    R = np.broadcast_to(np.eye(3), (t.size, 3, 3)).copy()
    d = np.zeros((t.size, 3))
    c = np.zeros(3)
    if spec.motion == 'velocity':
        d = t[:, None] * np.asarray(spec.velocity, dtype=np.float64)[None, :]
    elif spec.motion == 'rotation':
        c = np.asarray(spec.rot_centre, dtype=np.float64)
        a = spec.rot_omega * t
        ca, sa = np.cos(a), np.sin(a)
        R[:, 0, 0] = ca
        R[:, 0, 2] = -sa
        R[:, 2, 0] = sa
        R[:, 2, 2] = ca
    else:
        d = tissue_displacement(spec.motion, t)
    return R, d, c


def _apply_motion(p: np.ndarray, R: np.ndarray, d: np.ndarray, c: np.ndarray, motion: str) -> np.ndarray:
    """Positions at every frame: p [F][n][3] (tissue-frame positions per frame) or [1][n][3]."""
    if motion != 'rotation':
        return p + d[:, None, :]
    return c[None, None, :] + np.einsum('fij,fnj->fni', R, p - c[None, None, :]) + d[:, None, :]


def tissue_displacement(motion: str, t: np.ndarray) -> np.ndarray:
    """Rigid tissue displacement d(t), shape [len(t)][3] (metres)."""
    t = np.asarray(t, dtype=np.float64)
    d = np.zeros((t.size, 3))
    if motion == 'static':
        return d
    if motion == 'cardiac_resp':
        card = 100e-6 * np.sin(2 * np.pi * 1.0 * t)
        resp = 300e-6 * np.sin(2 * np.pi * 0.25 * t) / math.sqrt(2.0)
        d[:, 0] = resp
        d[:, 2] = card + resp
        return d
    if motion in ('velocity', 'rotation'):
        raise ValueError(f'motion {motion!r} is given by rigid_motion (it needs the scene spec)')
    raise ValueError(f'unknown motion {motion!r}')


def scene_box(cfg: Config):
    a, s = cfg.acq, cfg.scene
    (x0, y0, z0), (x1, y1, z1) = a.grid_box()
    lo = np.array([x0 - s.margin, y0 - s.margin, (z0 - s.margin) if s.z_lo is None else s.z_lo])
    hi = np.array([x1 + s.margin, y1 + s.margin, (z1 + s.margin) if s.z_hi is None else s.z_hi])
    return lo, hi


def _clip_line(c, u, lo, hi):
    """Parameter interval [s0, s1] of the line c + s u inside the box."""
    s0, s1 = -np.inf, np.inf
    for k in range(3):
        if abs(u[k]) < 1e-12:
            if c[k] < lo[k] or c[k] > hi[k]:
                return 0.0, 0.0
            continue
        a = (lo[k] - c[k]) / u[k]
        b = (hi[k] - c[k]) / u[k]
        s0, s1 = max(s0, min(a, b)), min(s1, max(a, b))
    return s0, max(s0, s1)


def _clipped_vessel(c, u, radius, vmax, lo, hi) -> Optional[Vessel]:
    s0, s1 = _clip_line(c, u, lo, hi)
    if s1 - s0 <= 2 * radius:
        return None
    return Vessel(centre=c + 0.5 * (s0 + s1) * u, axis=u, radius=radius,
                  half_len=0.5 * (s1 - s0), vmax=vmax)


def _unit(v):
    return v / np.linalg.norm(v)


def _random_dir(rng):
    while True:
        v = rng.normal(size=3)
        n = np.linalg.norm(v)
        if n > 1e-6:
            return v / n


def _make_vessels(cfg: Config, rng) -> List[Vessel]:
    a, s = cfg.acq, cfg.scene
    lo, hi = scene_box(cfg)
    glo, ghi = (np.array(p) for p in a.grid_box())
    gc = 0.5 * (glo + ghi)
    out: List[Vessel] = []
    if s.vessels == 'none':
        return out
    if s.vessels == 'one_45deg':
        v = _clipped_vessel(gc, _unit(np.array([1.0, 0.0, 1.0])), 0.5 * s.vessel_diam, s.vmax, lo, hi)
        return [v]
    if s.vessels == 'random3':
        q = 0.25 * (ghi - glo)
        while len(out) < 3:
            c = rng.uniform(glo + q, ghi - q)
            u = _random_dir(rng)
            diam = rng.uniform(0.2e-3, 1.0e-3)
            vmax = rng.uniform(5e-3, 30e-3)
            v = _clipped_vessel(c, u, 0.5 * diam, vmax, lo, hi)
            if v is not None:
                out.append(v)
        return out
    if s.vessels == 'murray31':
        return _murray_tree(glo, ghi, rng)
    raise ValueError(f'unknown vessel recipe {s.vessels!r}')


def _murray_tree(glo, ghi, rng) -> List[Vessel]:
    """5-generation binary tree (31 segments).  Murray's law r_p^3 = r_1^3 + r_2^3
    with a seeded asymmetric split, radii clamped to [50, 600] um, bifurcation
    angles U(35, 55) deg (Section 2.1.1), vmax proportional to radius (Poiseuille
    with Murray scaling), root 40 mm/s, clamped to [2, 40] mm/s."""
    ext = ghi - glo
    root_start = np.array([glo[0] + 0.5 * ext[0], glo[1] + 0.5 * ext[1], glo[2] + 0.05 * ext[2]])
    segs: List[Vessel] = []
    seg_len0 = 0.30 * ext[2]

    def grow(p0, u, r, gen, length):
        r = float(np.clip(r, 50e-6, 600e-6))
        p1 = p0 + length * u
        vmax = float(np.clip(40e-3 * r / 600e-6, 2e-3, 40e-3))
        segs.append(Vessel(centre=0.5 * (p0 + p1), axis=u, radius=r, half_len=0.5 * length, vmax=vmax))
        if gen == 4:
            return
        frac = rng.uniform(0.3, 0.7)
        r1, r2 = r * frac ** (1 / 3), r * (1 - frac) ** (1 / 3)
        beta = math.radians(rng.uniform(35.0, 55.0))
        w = _random_dir(rng)
        w = _unit(w - np.dot(w, u) * u)               # bifurcation plane normal to u
        for rr, sgn in ((r1, 1.0), (r2, -1.0)):
            d = _unit(math.cos(beta / 2) * u + sgn * math.sin(beta / 2) * w)
            grow(p1, d, rr, gen + 1, 0.72 * length)

    grow(root_start, np.array([0.0, 0.0, 1.0]), 600e-6, 0, seg_len0)
    return segs


def _inside_any(p: np.ndarray, vessels: List[Vessel]) -> np.ndarray:
    ins = np.zeros(p.shape[0], dtype=bool)
    for v in vessels:
        d = p - v.centre
        s = d @ v.axis
        r2 = np.einsum('ij,ij->i', d, d) - s * s
        ins |= (np.abs(s) <= v.half_len) & (r2 <= v.radius ** 2)
    return ins


def make_scene(cfg: Config, seed: Optional[int] = None) -> Scene:
    """Draw a scene.  Draw order (fixed): vessels, blood (axial, radial, angle),
    tissue positions (rejection outside the lumina), tissue amplitudes, blood amplitudes."""
    a, s = cfg.acq, cfg.scene
    rng = np.random.default_rng(s.seed if seed is None else seed)
    lo, hi = scene_box(cfg)
    vessels = _make_vessels(cfg, rng)
    F = a.n_frames
    times = np.arange(F, dtype=np.float64) / a.prf
    Rm, disp, cm = rigid_motion(s, times)                           # [F][3][3], [F][3], [3]

    # ---- blood: split by lumen volume, uniform in each lumen
    nb = s.n_blood if vessels else 0
    if nb:
        vol = np.array([v.half_len * v.radius ** 2 for v in vessels])
        counts = np.floor(nb * vol / vol.sum()).astype(int)
        counts[np.argmax(vol)] += nb - counts.sum()
    else:
        counts = np.zeros(len(vessels), dtype=int)
    bpos = np.zeros((F, nb, 3))
    bves = np.zeros(nb, dtype=np.int32)
    brad = np.zeros(nb)
    k = 0
    for iv, (v, n) in enumerate(zip(vessels, counts)):
        if n == 0:
            continue
        s0 = rng.uniform(-v.half_len, v.half_len, size=n)
        rr = v.radius * np.sqrt(rng.uniform(0.0, 1.0, size=n))
        ph = rng.uniform(0.0, 2 * np.pi, size=n)
        e1 = _unit(np.cross(v.axis, [1.0, 0.0, 0.0]) if abs(v.axis[0]) < 0.9
                   else np.cross(v.axis, [0.0, 1.0, 0.0]))
        e2 = np.cross(v.axis, e1)
        radial = (rr * np.cos(ph))[:, None] * e1 + (rr * np.sin(ph))[:, None] * e2
        speed = v.vmax * (1.0 - (rr / v.radius) ** 2)
        L = 2 * v.half_len
        sf = s0[None, :] + speed[None, :] * times[:, None]           # [F][n]
        sf = (sf + v.half_len) % L - v.half_len
        bpos[:, k:k + n, :] = _apply_motion(v.centre[None, None, :] + sf[:, :, None] * v.axis[None, None, :]
                                            + radial[None, :, :], Rm, disp, cm, s.motion)
        bves[k:k + n] = iv
        brad[k:k + n] = rr / v.radius
        k += n

    # ---- tissue: uniform in the box, outside every lumen
    nt = s.n_tissue
    tp = np.zeros((0, 3))
    while tp.shape[0] < nt:
        need = nt - tp.shape[0]
        cand = rng.uniform(lo, hi, size=(int(need * 1.1) + 16, 3))
        cand = cand[~_inside_any(cand, vessels)]
        tp = np.concatenate([tp, cand[:need]], axis=0)
    tamp = rng.normal(0.0, s.tissue_std, size=nt)
    bamp = rng.normal(0.0, s.blood_std, size=nb)
    if s.motion == 'static':
        tpos = tp[None, :, :]
    else:
        tpos = _apply_motion(np.broadcast_to(tp[None, :, :], (F,) + tp.shape), Rm, disp, cm, s.motion)
    return Scene(tissue_pos=np.ascontiguousarray(tpos, dtype=np.float32),
                 tissue_amp=tamp.astype(np.float32),
                 blood_pos=np.ascontiguousarray(bpos, dtype=np.float32),
                 blood_amp=bamp.astype(np.float32),
                 vessels=vessels, blood_vessel=bves, blood_radial=brad, times=times)


def point_scene(positions: np.ndarray, amps: np.ndarray) -> Scene:
    """A hand-placed scene: positions [F][S][3] (or [1][S][3]) and amplitudes [S]."""
    positions = np.asarray(positions, dtype=np.float32)
    F = positions.shape[0]
    return Scene(tissue_pos=positions, tissue_amp=np.asarray(amps, dtype=np.float32),
                 blood_pos=np.zeros((F, 0, 3), np.float32), blood_amp=np.zeros(0, np.float32),
                 vessels=[], blood_vessel=np.zeros(0, np.int32), blood_radial=np.zeros(0),
                 times=np.arange(F, dtype=np.float64))
