"""Acquisition and scene parameters of the synthetic workloads.

Workloads (all synthetic; no dataset is used):
  c1        16x16 array, 3 x-tilts, 32x32x64 voxels, 20 frames, static tissue,
            one 1 mm vessel.                         (small parity case)
  c2        32x32 array, 3x3 tilts, 128^3 voxels, 200 frames, moving tissue,
            three random vessels.                    (throughput workload)
  c3        = c2 (same seed); the split-BF16 Gram variant runs on it.
  c4_train  c2 acquisition on a 64^3 grid, scene scaled by volume; seeds
            1000-1063 give the learned filter's training pairs.
  c5        32x32 array, 9 tilts, 160x160x256 voxels, 400 frames at 2 kHz,
            31-segment bifurcating vessel tree.
  p7        the paper's DAS timing shape (Section 2.4.1): 32x32 active elements,
            7.81 MHz, 5 tilted plane waves, a 2 cm cube at 0.2 mm.

Grid convention: voxel centres r = (x0 + ix*dx, y0 + iy*dy, z0 + iz*dz),
linear voxel index v = ix + nx*(iy + ny*iz).  Lateral grids are centred on
the array axis.  Element e = ix + nx_el*iy sits at
((ix - (nx_el-1)/2)*pitch, (iy - (ny_el-1)/2)*pitch, 0).
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Tuple


@dataclasses.dataclass(frozen=True)
class Acq:
    """Acquisition: probe, transmits, voxel grid, slow time, RF record."""
    nx_el: int
    ny_el: int
    pitch: float                     # m
    fc: float                        # Hz, centre frequency
    fs: float                        # Hz, RF sampling rate
    c: float                         # m/s, speed of sound
    tilts_deg: Tuple[Tuple[float, float], ...]   # (theta_x, theta_y) per transmit
    nx: int
    ny: int
    nz: int
    dx: float
    dy: float
    dz: float
    z0: float                        # depth of the first voxel plane, m
    n_frames: int
    prf: float                       # Hz, frame (ensemble) rate
    n_samples: int                   # RF samples per trace

    @property
    def n_elem(self) -> int:
        return self.nx_el * self.ny_el

    @property
    def n_angles(self) -> int:
        return len(self.tilts_deg)

    @property
    def n_vox(self) -> int:
        return self.nx * self.ny * self.nz

    @property
    def x0(self) -> float:
        return -0.5 * (self.nx - 1) * self.dx

    @property
    def y0(self) -> float:
        return -0.5 * (self.ny - 1) * self.dy

    @property
    def wavelength(self) -> float:
        return self.c / self.fc

    def tilts_rad(self) -> List[Tuple[float, float]]:
        return [(math.radians(a), math.radians(b)) for a, b in self.tilts_deg]

    def grid_box(self):
        """(lo, hi) corners of the voxel-centre box."""
        lo = (self.x0, self.y0, self.z0)
        hi = (self.x0 + (self.nx - 1) * self.dx, self.y0 + (self.ny - 1) * self.dy,
              self.z0 + (self.nz - 1) * self.dz)
        return lo, hi

    def das_units(self) -> int:
        """voxel x element x angle x frame products of one beamformed ensemble."""
        return self.n_vox * self.n_elem * self.n_angles * self.n_frames

    def with_(self, **kw) -> "Acq":
        return dataclasses.replace(self, **kw)


@dataclasses.dataclass(frozen=True)
class SceneSpec:
    """Scatterer scene recipe (positions are drawn by scene.make_scene)."""
    n_tissue: int
    tissue_std: float                # tissue reflectivity ~ N(0, tissue_std)
    n_blood: int
    blood_std: float                 # blood reflectivity ~ N(0, blood_std)
    vessels: str                     # 'one_45deg' | 'random3' | 'murray31' | 'none'
    vessel_diam: float = 1e-3        # 'one_45deg': lumen diameter, m
    vmax: float = 20e-3              # 'one_45deg': centre-line speed, m/s
    motion: str = 'static'           # 'static' | 'cardiac_resp' | 'velocity' | 'rotation'
    z_lo: Optional[float] = None     # scene depth range; default grid depth +- margin
    z_hi: Optional[float] = None
    margin: float = 1e-3             # lateral (and default depth) margin around the grid
    seed: int = 0
    velocity: Tuple[float, float, float] = (0.0, 0.0, 0.0)   # 'velocity': m/s
    rot_omega: float = 0.0           # 'rotation': rad/s about -y (angular velocity (0, -w, 0))
    rot_centre: Tuple[float, float, float] = (0.0, 0.0, 0.025)   # 'rotation': m


@dataclasses.dataclass(frozen=True)
class Config:
    name: str
    acq: Acq
    scene: SceneSpec
    cutoff: int                      # >= 0 fixed clutter rank, -1 = knee rule


C_SOUND = 1540.0
FC = 7.8e6
FS = 31.25e6
HALF_LAMBDA = 0.5 * C_SOUND / FC


def _acq(nx_el, ny_el, tilts, nx, ny, nz, n_frames, prf, n_samples,
         fc=FC, fs=FS, pitch=0.3e-3, spacing=None, z0=5e-3):
    d = HALF_LAMBDA if spacing is None else spacing
    return Acq(nx_el=nx_el, ny_el=ny_el, pitch=pitch, fc=fc, fs=fs, c=C_SOUND,
               tilts_deg=tuple(tilts), nx=nx, ny=ny, nz=nz, dx=d, dy=d, dz=d,
               z0=z0, n_frames=n_frames, prf=prf, n_samples=n_samples)


_T3X = ((-5.0, 0.0), (0.0, 0.0), (5.0, 0.0))
_T9 = tuple((a, b) for b in (-6.0, 0.0, 6.0) for a in (-6.0, 0.0, 6.0))
_T5 = ((0.0, 0.0), (-5.0, 0.0), (5.0, 0.0), (0.0, -5.0), (0.0, 5.0))

# RF record lengths: the longest two-way path in each scene box plus the pulse
# half-length and a guard, rounded up to a multiple of 128 samples.
CONFIGS = {
    'c1': Config('c1', _acq(16, 16, _T3X, 32, 32, 64, 20, 1000.0, 768),
                 SceneSpec(n_tissue=2000, tissue_std=1.0, n_blood=500, blood_std=0.1,
                           vessels='one_45deg', vessel_diam=1e-3, vmax=20e-3,
                           motion='static', z_lo=5e-3, z_hi=15e-3, seed=1),
                 cutoff=2),
    'c2': Config('c2', _acq(32, 32, _T9, 128, 128, 128, 200, 1000.0, 1024),
                 SceneSpec(n_tissue=50000, tissue_std=1.0, n_blood=20000, blood_std=0.01,
                           vessels='random3', motion='cardiac_resp', seed=2),
                 cutoff=-1),
    'c4_train': Config('c4_train', _acq(32, 32, _T9, 64, 64, 64, 200, 1000.0, 768),
                       SceneSpec(n_tissue=6250, tissue_std=1.0, n_blood=2500, blood_std=0.01,
                                 vessels='random3', motion='cardiac_resp', seed=1000),
                       cutoff=-1),
    'c5': Config('c5', _acq(32, 32, _T9, 160, 160, 256, 400, 2000.0, 1536),
                 SceneSpec(n_tissue=200000, tissue_std=1.0, n_blood=30000, blood_std=0.01,
                           vessels='murray31', motion='cardiac_resp', seed=5),
                 cutoff=-1),
    'p7': Config('p7', _acq(32, 32, _T5, 100, 100, 100, 30, 1000.0, 1408, fc=7.81e6,
                            spacing=0.2e-3),
                 SceneSpec(n_tissue=50000, tissue_std=1.0, n_blood=20000, blood_std=0.01,
                           vessels='random3', motion='cardiac_resp', seed=7),
                 cutoff=-1),
}
CONFIGS['c3'] = dataclasses.replace(CONFIGS['c2'], name='c3')
# small learned-filter case for tests: the small array and transmits, a 32^3 grid, 64
# frames, moving tissue and three random vessels (the throughput workload's scene recipe)
CONFIGS['c4_small'] = Config('c4_small', _acq(16, 16, _T3X, 32, 32, 32, 64, 1000.0, 512),
                             SceneSpec(n_tissue=3000, tissue_std=1.0, n_blood=1500, blood_std=0.01,
                                       vessels='random3', motion='cardiac_resp', seed=2000),
                             cutoff=-1)


def get_config(name: str) -> Config:
    return CONFIGS[name]


# Tissue-motion sweep (the synthetic analog of the motion study of Section 3): steady
# axial motion V_z = 2, 4, 8 mm/s; lateral V_x = 2, 4, 8 mm/s at V_z = 4 mm/s; rotation
# V = (0, -w, 0) x (r - (0, 0, 2.5 cm)) with w = 1 rad/s scaled by 0.1, 0.2, 0.4.  Vessels
# move with the tissue.  Geometry of the training workload (64^3, 9 transmits, 200 frames).
MOTION_SWEEP = (
    ('vz2', dict(motion='velocity', velocity=(0.0, 0.0, 2e-3))),
    ('vz4', dict(motion='velocity', velocity=(0.0, 0.0, 4e-3))),
    ('vz8', dict(motion='velocity', velocity=(0.0, 0.0, 8e-3))),
    ('vx2_vz4', dict(motion='velocity', velocity=(2e-3, 0.0, 4e-3))),
    ('vx4_vz4', dict(motion='velocity', velocity=(4e-3, 0.0, 4e-3))),
    ('vx8_vz4', dict(motion='velocity', velocity=(8e-3, 0.0, 4e-3))),
    ('rot0.1', dict(motion='rotation', rot_omega=0.1)),
    ('rot0.2', dict(motion='rotation', rot_omega=0.2)),
    ('rot0.4', dict(motion='rotation', rot_omega=0.4)),
)


def augmented_motion_config(base: str, seed: int) -> Config:
    """The base workload with a seeded steady tissue motion, for training data that spans
    the motion sweep's range: even seeds a constant velocity (0.5-10 mm/s, uniform
    direction), odd seeds a rotation about -y (0.05-0.5 rad/s about a centre 15-35 mm
    deep).  The scene itself is drawn with the same seed."""
    import numpy as np
    b = CONFIGS[base]
    rng = np.random.default_rng(seed + 7_777_777)
    if seed % 2 == 0:
        d = rng.standard_normal(3)
        d /= np.linalg.norm(d)
        v = tuple(float(x) for x in d * rng.uniform(0.5e-3, 10e-3))
        sc = dataclasses.replace(b.scene, seed=seed, motion='velocity', velocity=v)
    else:
        sc = dataclasses.replace(b.scene, seed=seed, motion='rotation', rot_omega=float(rng.uniform(0.05, 0.5)),
                                 rot_centre=(0.0, 0.0, float(rng.uniform(15e-3, 35e-3))))
    return dataclasses.replace(b, name=f'{base}_aug{seed}', scene=sc)


def motion_sweep_configs(base: str = 'c4_train', seed: int = 3000) -> dict:
    """name -> Config of the motion sweep, one seeded scene recipe for every case."""
    b = CONFIGS[base]
    return {name: dataclasses.replace(b, name=f'sweep_{name}',
                                      scene=dataclasses.replace(b.scene, seed=seed, **kw))
            for name, kw in MOTION_SWEEP}


def scaled(cfg: Config, *, frames: Optional[int] = None, seed: Optional[int] = None,
           n_tissue: Optional[int] = None, n_blood: Optional[int] = None) -> Config:
    """Same acquisition geometry with fewer frames / another seed / scatterer count."""
    acq = cfg.acq if frames is None else cfg.acq.with_(n_frames=frames)
    sc = cfg.scene
    kw = {}
    if seed is not None:
        kw['seed'] = seed
    if n_tissue is not None:
        kw['n_tissue'] = n_tissue
    if n_blood is not None:
        kw['n_blood'] = n_blood
    if kw:
        sc = dataclasses.replace(sc, **kw)
    return dataclasses.replace(cfg, acq=acq, scene=sc)
