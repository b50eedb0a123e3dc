"""Synthetic street corridors standing in for the paper's driving datasets.

The paper evaluates on recorded driving sequences (Sec. 4.1, "Datasets"); those
are not available here, so every workload is drawn from a seeded generator with
the structure of a street scene: a long static corridor whose density decays away
from the road centreline, a set of rigid dynamic instances moving on smooth SE(3)
tracks, and a forward camera (or a 6-camera surround rig) driving along the
centreline.  Nothing here reproduces any item of those datasets.

Frames.  World: x along the road, y to the left, z up, ground at z = 0.
Camera: OpenCV convention (x right, y down, z forward).  A camera extrinsic is
the 3x4 world->camera matrix [R | t]; an instance pose is the 3x4 local->world
matrix [R_G | t_G] of that instance at one timestep (slot 0 of every timestep is
the identity and stands for the static background).

Attribute conventions consumed by the renderer:
  mean    (N,3) f32  position; instance-local for instance Gaussians
  scale   (N,3) f32  per-axis standard deviation in metres (already activated)
  quat    (N,4) f32  rotation quaternion (w, x, y, z), *not* normalised
  opacity (N,)  f32  in (0, 1) (already activated)
  sh      (N,B,3) f32 real-SH colour coefficients, B = (L+1)^2
  inst    (N,)  i32  0 = static, k in 1..K = instance k
  vis_s, vis_e (N,) f32   temporal visibility, initial (-1, 1)
  life_s, life_e (N,) f32 point life, initial (1, -1)
Static Gaussians come first, sorted along the road (x ascending), then each
instance's Gaussians contiguously.
"""

from __future__ import annotations

import math
from dataclasses import dataclass, field, replace

import numpy as np

SEED_BASE = 250308217


# --------------------------------------------------------------------------
# containers
# --------------------------------------------------------------------------
@dataclass
class Scene:
    mean: np.ndarray
    scale: np.ndarray
    quat: np.ndarray
    opacity: np.ndarray
    sh: np.ndarray
    inst: np.ndarray
    vis_s: np.ndarray
    vis_e: np.ndarray
    life_s: np.ndarray
    life_e: np.ndarray
    pose: np.ndarray  # (T, K+1, 3, 4) f32 local->world, slot 0 identity
    sh_degree: int

    @property
    def n(self) -> int:
        return int(self.mean.shape[0])

    @property
    def n_slots(self) -> int:  # K + 1
        return int(self.pose.shape[1])

    @property
    def n_timesteps(self) -> int:
        return int(self.pose.shape[0])

    def copy(self) -> "Scene":
        return replace(self, **{k: np.array(getattr(self, k)) for k in (
            "mean", "scale", "quat", "opacity", "sh", "inst", "vis_s", "vis_e",
            "life_s", "life_e", "pose")})


@dataclass
class Views:
    W: np.ndarray      # (V, 3, 4) f32 world->camera
    K: np.ndarray      # (V, 4) f32 fx, fy, cx, cy
    wh: np.ndarray     # (V, 2) i32 width, height
    tstep: np.ndarray  # (V,) i32 timestep index tau in [0, T)

    @property
    def n_views(self) -> int:
        return int(self.W.shape[0])

    def subset(self, idx) -> "Views":
        idx = np.asarray(idx)
        return Views(self.W[idx].copy(), self.K[idx].copy(), self.wh[idx].copy(),
                     self.tstep[idx].copy())


@dataclass
class Config:
    cfg: int
    name: str
    scene: Scene
    views: Views
    params: dict
    timed_views: list = field(default_factory=list)
    warmup_fold: bool = False


def default_params(**over) -> dict:
    """Renderer constants.  Values the paper leaves open are the 3DGS ones."""
    p = dict(
        tile=16,
        lod_r=0.0,         # LOD threshold in pixels (0 disables the cull)
        z_near=0.2,
        z_far=float("inf"),
        eps2d=0.3,         # screen-space low-pass added to the 2D covariance
        alpha_min=1.0 / 255.0,
        alpha_max=0.99,
        t_min=1e-4,
        cutoff=4.5,        # Mahalanobis cut (-power > cutoff => skip)
        jac_clamp=1.3,
        bg=(0.0, 0.0, 0.0),
        temporal=False,
        lod=False,
        margin=0.1,        # FOLD margin of the temporal-visibility update
    )
    p.update(over)
    return p


# --------------------------------------------------------------------------
# input construction helpers (frames only; no rendering arithmetic)
# --------------------------------------------------------------------------
def _rot_zyx(yaw, pitch, roll):
    cy, sy = math.cos(yaw), math.sin(yaw)
    cp, sp = math.cos(pitch), math.sin(pitch)
    cr, sr = math.cos(roll), math.sin(roll)
    rz = np.array([[cy, -sy, 0], [sy, cy, 0], [0, 0, 1]], np.float64)
    ry = np.array([[cp, 0, sp], [0, 1, 0], [-sp, 0, cp]], np.float64)
    rx = np.array([[1, 0, 0], [0, cr, -sr], [0, sr, cr]], np.float64)
    return rz @ ry @ rx


def _camera(pos, yaw):
    """World->camera extrinsic of a level OpenCV camera at `pos` heading `yaw`."""
    f = np.array([math.cos(yaw), math.sin(yaw), 0.0])
    r = np.array([math.sin(yaw), -math.cos(yaw), 0.0])
    d = np.array([0.0, 0.0, -1.0])
    R = np.stack([r, d, f])
    t = -R @ np.asarray(pos, np.float64)
    return np.concatenate([R, t[:, None]], axis=1)


def _fx_for_hfov(width, hfov_deg=70.0):
    return (0.5 * width) / math.tan(math.radians(0.5 * hfov_deg))


def _attrs(rng, n, sh_degree, sh_sigma):
    scale = np.exp(rng.normal(math.log(0.05), 0.5, size=(n, 3)))
    q = rng.normal(size=(n, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    q *= rng.uniform(0.5, 1.5, size=(n, 1))  # unnormalised on purpose
    opac = 1.0 / (1.0 + np.exp(-rng.normal(size=n)))
    nb = (sh_degree + 1) ** 2
    if sh_degree == 0:
        rgb = rng.uniform(0.0, 1.0, size=(n, 3))
        sh = ((rgb - 0.5) * (2.0 * math.sqrt(math.pi)))[:, None, :]
    else:
        sh = rng.normal(0.0, sh_sigma, size=(n, nb, 3))
    return (scale.astype(np.float32), q.astype(np.float32),
            opac.astype(np.float32), sh.astype(np.float32))


def _corridor_static(rng, n, length, half_width=20.0, height=10.0, mean_off=8.0):
    """Static points: uniform along x, |y| ~ Exp(mean_off) truncated, z uniform."""
    x = rng.uniform(0.0, length, size=n)
    u = rng.uniform(0.0, 1.0, size=n)
    a = 1.0 - math.exp(-half_width / mean_off)
    ay = -mean_off * np.log1p(-u * a)          # truncated exponential
    y = ay * rng.choice([-1.0, 1.0], size=n)
    z = rng.uniform(0.0, height, size=n)
    xyz = np.stack([x, y, z], axis=1)
    # stored in corridor order (ascending x): Gaussians seen over the same
    # stretch of the drive are neighbours in memory
    return xyz[np.argsort(x, kind="stable")]


def _assemble(rng, static_xyz, inst_local, sh_degree, sh_sigma, poses):
    n_s = static_xyz.shape[0]
    means = [static_xyz] + inst_local
    mean = np.concatenate(means, axis=0).astype(np.float32)
    inst = np.concatenate([np.zeros(n_s, np.int32)] +
                          [np.full(m.shape[0], k + 1, np.int32)
                           for k, m in enumerate(inst_local)])
    n = mean.shape[0]
    scale, quat, opac, sh = _attrs(rng, n, sh_degree, sh_sigma)
    return Scene(
        mean=mean, scale=scale, quat=quat, opacity=opac, sh=sh, inst=inst,
        vis_s=np.full(n, -1.0, np.float32), vis_e=np.full(n, 1.0, np.float32),
        life_s=np.full(n, 1.0, np.float32), life_e=np.full(n, -1.0, np.float32),
        pose=poses.astype(np.float32), sh_degree=sh_degree)


def _tracks(rng, K, T, x_lo, x_hi, box_h=1.5):
    """Smooth SE(3) tracks: forward motion at 5-15 m/s (10 Hz), lane wobble,
    yaw along the velocity, small roll/pitch oscillation."""
    poses = np.zeros((T, K + 1, 3, 4), np.float64)
    poses[:, 0, :, :3] = np.eye(3)
    x0 = rng.uniform(x_lo, x_hi, size=K)
    lane = rng.uniform(-6.0, 6.0, size=K)
    speed = rng.uniform(5.0, 15.0, size=K)
    phase = rng.uniform(0.0, 2 * math.pi, size=K)
    for k in range(K):
        for tau in range(T):
            w = 2 * math.pi / max(T, 1)
            x = x0[k] + speed[k] * 0.1 * tau
            y = lane[k] + 0.5 * math.sin(w * tau + phase[k])
            vx = speed[k] * 0.1
            vy = 0.5 * w * math.cos(w * tau + phase[k])
            yaw = math.atan2(vy, vx)
            wob = 0.02 * math.sin(w * tau + phase[k])
            poses[tau, k + 1, :, :3] = _rot_zyx(yaw, wob, wob)
            poses[tau, k + 1, :, 3] = (x, y, 0.5 * box_h)
    return poses


def _box(rng, n, hx, hy, hz):
    return np.stack([rng.uniform(-hx, hx, n), rng.uniform(-hy, hy, n),
                     rng.uniform(-hz, hz, n)], axis=1)


def _forward_views(T, x_end, width, height, taus, cam_h=1.6):
    f = _fx_for_hfov(width)
    W, K, wh, ts = [], [], [], []
    for tau in taus:
        x = x_end * tau / max(T - 1, 1)
        W.append(_camera((x, 0.0, cam_h), 0.0))
        K.append((f, f, 0.5 * width, 0.5 * height))
        wh.append((width, height))
        ts.append(tau)
    return Views(np.asarray(W, np.float32), np.asarray(K, np.float32),
                 np.asarray(wh, np.int32), np.asarray(ts, np.int32))


RIG = [  # (yaw degrees, width, height)
    (0.0, 1920, 1080),
    (60.0, 1550, 2048), (-60.0, 1550, 2048),
    (120.0, 2048, 1550), (-120.0, 2048, 1550),
    (180.0, 2048, 1550),
]


def _rig_views(T, x_end, taus, rig, cam_h=1.6):
    W, K, wh, ts = [], [], [], []
    for tau in taus:
        x = x_end * tau / max(T - 1, 1)
        for yaw_deg, w, h in rig:
            f = _fx_for_hfov(w)
            W.append(_camera((x, 0.0, cam_h), math.radians(yaw_deg)))
            K.append((f, f, 0.5 * w, 0.5 * h))
            wh.append((w, h))
            ts.append(tau)
    return Views(np.asarray(W, np.float32), np.asarray(K, np.float32),
                 np.asarray(wh, np.int32), np.asarray(ts, np.int32))


# --------------------------------------------------------------------------
# the five workloads
# --------------------------------------------------------------------------
def make_config(cfg: int, *, scale_n: float = 1.0) -> Config:
    """Build workload `cfg` (1..5).  `scale_n` shrinks every Gaussian count
    (used for quick tests of the larger shapes); 1.0 is the real size."""
    rng = np.random.default_rng(SEED_BASE + cfg)

    def sn(n):
        return max(1, int(round(n * scale_n)))

    if cfg == 1:
        static = np.stack([rng.uniform(4, 24, sn(2000)), rng.uniform(-4, 4, sn(2000)),
                           rng.uniform(-1.5, 1.5, sn(2000))], axis=1)
        local = _box(rng, sn(200), 2.0, 1.0, 0.75)
        T = 3
        poses = np.zeros((T, 2, 3, 4))
        poses[:, 0, :, :3] = np.eye(3)
        yaw = math.atan2(2.0, 2.0)
        for tau in range(T):
            poses[tau, 1, :, :3] = _rot_zyx(yaw, 0.0, 0.0)
            poses[tau, 1, :, 3] = (10.0 + 2.0 * tau, -2.0 + 2.0 * tau, 0.0)
        scene = _assemble(rng, static, [local], 0, 0.0, poses)
        W = np.asarray([_camera((0, 0, 0), 0.0)] * 3, np.float32)
        views = Views(W, np.asarray([(64, 64, 32, 32)] * 3, np.float32),
                      np.asarray([(64, 64)] * 3, np.int32), np.arange(3, dtype=np.int32))
        params = default_params(tile=16, lod_r=0.0, temporal=False, lod=False)
        return Config(1, "tiny-2.2k-64x64-3views", scene, views, params, [0, 1, 2])

    if cfg == 2:
        T = 50
        static = _corridor_static(rng, sn(200_000), 200.0)
        K = 8
        local = [_box(rng, sn(5_000), 2.25, 1.0, 0.75) for _ in range(K)]
        poses = _tracks(rng, K, T, 10.0, 120.0)
        scene = _assemble(rng, static, local, 3, 0.1, poses)
        views = _forward_views(T, 160.0, 960, 640, range(T))
        params = default_params(tile=16, lod_r=1.0, temporal=True, lod=True)
        return Config(2, "corridor-240k-960x640", scene, views, params, list(range(T)))

    if cfg == 3:
        T = 50
        static = _corridor_static(rng, sn(1_700_000), 1000.0)
        K = 30
        local = [_box(rng, sn(10_000), 2.25, 1.0, 0.75) for _ in range(K)]
        poses = _tracks(rng, K, T, 10.0, 900.0)
        scene = _assemble(rng, static, local, 3, 0.1, poses)
        views = _forward_views(T, 950.0, 1920, 1080, range(T))
        params = default_params(tile=16, lod_r=1.0, temporal=True, lod=True)
        timed = [int(round(i * (T - 1) / 7)) for i in range(8)]
        return Config(3, "corridor-2M-1080p", scene, views, params, timed, warmup_fold=True)

    if cfg == 4:
        T = 50
        static = _corridor_static(rng, sn(2_600_000), 1500.0)
        K = 40
        local = [_box(rng, sn(10_000), 2.25, 1.0, 0.75) for _ in range(K)]
        poses = _tracks(rng, K, T, 10.0, 1400.0)
        scene = _assemble(rng, static, local, 3, 0.1, poses)
        views = _rig_views(T, 1450.0, range(T), RIG)
        params = default_params(tile=16, lod_r=1.0, temporal=True, lod=True)
        timed = [i for i in range(views.n_views) if 20 <= views.tstep[i] <= 23]
        return Config(4, "rig-3M-24views", scene, views, params, timed, warmup_fold=True)

    if cfg == 5:
        T = 150
        static = _corridor_static(rng, sn(9_000_000), 3000.0)
        K = 100
        local = [_box(rng, sn(10_000), 2.25, 1.0, 0.75) for _ in range(K)]
        poses = _tracks(rng, K, T, 10.0, 2900.0)
        scene = _assemble(rng, static, local, 3, 0.1, poses)
        rig1080 = [(yaw, 1920, 1080) for yaw, _, _ in RIG]
        views = _rig_views(T, 2950.0, range(T), rig1080)
        params = default_params(tile=16, lod_r=1.0, temporal=True, lod=True, z_far=150.0)
        timed = [i for i in range(views.n_views) if 70 <= views.tstep[i] <= 73]
        return Config(5, "city-10M-24views", scene, views, params, timed, warmup_fold=True)

    raise ValueError(f"unknown config {cfg}")


def make_scaleup(length_m: float, *, density: float = 1700.0, inst_per_km: float = 30.0,
                 spacing_m: float = 20.0, scale_n: float = 1.0) -> Config:
    """Corridors of growing length at the mid corridor's density and camera
    (1700 static Gaussians per metre, 30 instances of 10k per km, one 1920x1080
    frame every `spacing_m` metres): the per-view cost as the scene grows,
    the paper's scale-up experiment with synthetic streets."""
    L = float(length_m)
    rng = np.random.default_rng(SEED_BASE + 600 + int(round(L)))
    T = max(2, int(round(L / spacing_m)))
    static = _corridor_static(rng, max(1, int(round(density * L * scale_n))), L)
    K = max(1, int(round(inst_per_km * L / 1000.0)))
    local = [_box(rng, max(1, int(round(10_000 * scale_n))), 2.25, 1.0, 0.75) for _ in range(K)]
    x_end = max(L - 50.0, 0.5 * L)
    poses = _tracks(rng, K, T, min(10.0, 0.1 * L), max(x_end - 50.0, 0.2 * L))
    scene = _assemble(rng, static, local, 3, 0.1, poses)
    views = _forward_views(T, x_end, 1920, 1080, range(T))
    params = default_params(tile=16, lod_r=1.0, temporal=True, lod=True)
    timed = sorted(set(int(round(i * (T - 1) / 7)) for i in range(8)))
    return Config(100 + int(round(L)), f"scaleup-{int(round(L))}m", scene, views, params, timed,
                  warmup_fold=True)


def micro_scene(seed: int, n: int = 8, width: int = 24, height: int = 20,
                n_inst: int = 1, sh_degree: int = 1, T: int = 2,
                spread: float = 1.0):
    """A handful of Gaussians in front of a small camera; used by property tests."""
    rng = np.random.default_rng(SEED_BASE + 77_000 + seed)
    n_dyn = n // 3 if n_inst > 0 else 0
    n_s = n - n_dyn
    static = np.stack([rng.uniform(3, 6, n_s), rng.uniform(-spread, spread, n_s),
                       rng.uniform(-spread, spread, n_s)], axis=1)
    locs = []
    if n_inst > 0:
        per = np.array_split(np.arange(n_dyn), n_inst)
        locs = [_box(rng, len(p), 0.5, 0.5, 0.5) for p in per]
    poses = np.zeros((T, n_inst + 1, 3, 4))
    poses[:, 0, :, :3] = np.eye(3)
    for k in range(n_inst):
        for tau in range(T):
            poses[tau, k + 1, :, :3] = _rot_zyx(rng.uniform(-0.5, 0.5), rng.uniform(-0.2, 0.2),
                                                rng.uniform(-0.2, 0.2))
            poses[tau, k + 1, :, 3] = (rng.uniform(3.5, 5), rng.uniform(-0.5, 0.5),
                                       rng.uniform(-0.5, 0.5))
    scene = _assemble(rng, static, locs, sh_degree, 0.3, poses)
    scene.scale[:] = np.exp(rng.normal(math.log(0.3), 0.4, size=(n, 3))).astype(np.float32)
    scene.opacity[:] = rng.uniform(0.2, 0.9, n).astype(np.float32)
    f = 0.9 * width
    W = [_camera((0, 0, 0), 0.0) for _ in range(T)]
    views = Views(np.asarray(W, np.float32),
                  np.asarray([(f, f, 0.5 * width, 0.5 * height)] * T, np.float32),
                  np.asarray([(width, height)] * T, np.int32), np.arange(T, dtype=np.int32))
    return scene, views


def targets(cfg: int, views: Views, view_ids=None):
    """Seeded U(0,1) targets, one (3, H, W) f32 image per view."""
    ids = range(views.n_views) if view_ids is None else view_ids
    out = []
    for v in ids:
        w, h = int(views.wh[v, 0]), int(views.wh[v, 1])
        rng = np.random.default_rng(SEED_BASE + 1000 * cfg + int(v))
        out.append(rng.uniform(0.0, 1.0, size=(3, h, w)).astype(np.float32))
    return out
