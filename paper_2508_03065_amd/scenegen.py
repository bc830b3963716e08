"""Seeded synthetic scenes for moving-source image-source synthesis.

This module only *describes* inputs: rooms, wall coefficients, trajectories,
microphone offsets, source signals and synthesis parameters.  It holds none of
the synthesis arithmetic (no image enumeration, delays, gains or filters), so
both the GPU library binding and the CPU oracle may consume its output.

The workloads mirror the paper's setting (Sec. III: 16 kHz speech-rate audio,
moving talkers, reverberant rooms with reflection orders into the tens; the
Sec. II-C example of a T60 = 0.6 s room).  The paper's speech and noise corpora
are not available, so the source signal is seeded i.i.d. N(0, 1) noise, a
full-band stand-in that is stricter than speech for the fractional-delay filter.
"""
from __future__ import annotations

import dataclasses
import math
from dataclasses import dataclass, field
from typing import List, Optional, Sequence, Tuple

import numpy as np

PWL = 0
CIRCLE = 1


@dataclass
class Traj:
    """A trajectory: piecewise linear through knots (clamped outside the knot
    range; one knot = static) or a horizontal circle."""
    kind: int = PWL
    t: np.ndarray = field(default_factory=lambda: np.zeros(1))
    p: np.ndarray = field(default_factory=lambda: np.zeros((1, 3)))
    center: Tuple[float, float, float] = (0.0, 0.0, 0.0)
    radius: float = 0.0
    speed: float = 0.0
    phase0: float = 0.0

    @staticmethod
    def static(pos) -> "Traj":
        return Traj(PWL, np.zeros(1), np.asarray(pos, dtype=np.float64).reshape(1, 3))

    @staticmethod
    def pwl(t, p) -> "Traj":
        return Traj(PWL, np.asarray(t, dtype=np.float64), np.asarray(p, dtype=np.float64).reshape(-1, 3))

    @staticmethod
    def circle(center, radius, speed, phase0=0.0) -> "Traj":
        return Traj(CIRCLE, np.zeros(1), np.zeros((1, 3)), tuple(float(v) for v in center),
                    float(radius), float(speed), float(phase0))

    def copy(self) -> "Traj":
        return dataclasses.replace(self, t=self.t.copy(), p=self.p.copy())


@dataclass
class Scene:
    size: np.ndarray              # (3,) room Lx, Ly, Lz in m
    beta: np.ndarray              # (6,) walls x=0, x=Lx, y=0, y=Ly, z=0, z=Lz
    src: Traj
    rcv: Traj
    mic_offset: np.ndarray        # (C, 3) offsets from the receiver point
    x: np.ndarray                 # (n_in,) float32 source signal
    n_out: int
    max_order: int                # K for this scene

    @property
    def n_in(self) -> int:
        return int(self.x.shape[0])

    @property
    def n_mics(self) -> int:
        return int(self.mic_offset.shape[0])

    def copy(self) -> "Scene":
        return Scene(self.size.copy(), self.beta.copy(), self.src.copy(), self.rcv.copy(),
                     self.mic_offset.copy(), self.x.copy(), self.n_out, self.max_order)


@dataclass
class Params:
    c: float = 343.0
    fs: float = 16000.0
    taps: int = 64
    kaiser_beta: float = 8.0
    cutoff: float = 0.5
    tiers: Tuple[Tuple[int, int], ...] = ()   # ((max_order, decimation), ...); () = full rate
    delay_model: int = 0                      # 0 retarded, 1 instantaneous
    fd_kind: int = 0                          # how the library applies the kernel: 0 table, 1 Farrow
    farrow_order: int = 9
    knot_slack: float = 0.0                   # m a plan lets its source knots move (msim_plan_update)
    tier_mode: int = 0                        # 0: tiers by order; 1: adaptive per image (tier_tol, tier_rmax)
    tier_tol: float = 1e-3                    # adaptive: delay interpolation error bound, samples
    tier_rmax: int = 1024                     # adaptive: largest decimation
    adjx_mode: int = 0                        # dL/dx: 0 Farrow gather, 1 the table form's own transpose


PAPER_TIERS = ((2, 1), (6, 16), (1 << 20, 160))


def n_out_for(size, max_order: int, n_in: int, fs: float, c: float, taps: int) -> int:
    """Output length that holds every contribution: n_in + ceil(fs*d_max/c) + T.

    d_max bounds the distance between any point of the room and any point of an
    image cell |m|_1 <= K: per axis at most L_a(|m_a|+1); the sum of squares is
    largest with the whole order on the longest axis."""
    L = sorted(float(v) for v in size)
    d2 = (L[2] * (max_order + 1)) ** 2 + L[1] ** 2 + L[0] ** 2
    return int(n_in + math.ceil(fs * math.sqrt(d2) / c) + taps)


def noise(rng: np.random.Generator, n: int) -> np.ndarray:
    return rng.standard_normal(n).astype(np.float32)


def _inside(p, size, margin):
    return all(margin <= p[a] <= size[a] - margin for a in range(3))


def random_pwl(rng, size, n_knots, duration, speed_lo, speed_hi, margin=0.5,
               start=None, keep_away=None, min_sep=0.5, planar=False) -> Traj:
    """Straight segments of random direction and speed between n_knots knots
    spread evenly over [0, duration]; every knot stays inside the room with a
    wall margin (directions are redrawn, then speeds shrunk, until it does)."""
    size = np.asarray(size, dtype=np.float64)
    lo, hi = np.full(3, margin), size - margin
    if start is None:
        for _ in range(1000):
            start = rng.uniform(lo, hi)
            if keep_away is None or np.linalg.norm(start - keep_away) >= min_sep:
                break
    pts = [np.asarray(start, dtype=np.float64)]
    ts = np.linspace(0.0, duration, n_knots)
    for k in range(1, n_knots):
        dt = ts[k] - ts[k - 1]
        v = rng.uniform(speed_lo, speed_hi)
        nxt = None
        for attempt in range(400):
            d = rng.standard_normal(3)
            if planar:
                d[2] = 0.0
            d /= np.linalg.norm(d)
            scale = 1.0 if attempt < 200 else 0.5 ** ((attempt - 199) / 20.0)
            cand = pts[-1] + d * v * scale * dt
            if _inside(cand, size, margin) and (keep_away is None or np.linalg.norm(cand - keep_away) >= min_sep):
                nxt = cand
                break
        if nxt is None:
            nxt = pts[-1].copy()
        pts.append(nxt)
    return Traj.pwl(ts, np.stack(pts))


def random_circle(rng, size, speed_lo, speed_hi, r_lo=0.5, r_hi=2.0, margin=0.5, h_lo=1.0, h_hi=2.0) -> Traj:
    size = np.asarray(size, dtype=np.float64)
    r_max = 0.5 * min(size[0], size[1]) - margin - 1e-3
    R = float(np.clip(rng.uniform(r_lo, r_hi), 0.1, r_max))
    cx = rng.uniform(margin + R, size[0] - margin - R)
    cy = rng.uniform(margin + R, size[1] - margin - R)
    h = float(np.clip(rng.uniform(h_lo, h_hi), margin, size[2] - margin))
    return Traj.circle((cx, cy, h), R, rng.uniform(speed_lo, speed_hi), rng.uniform(0, 2 * math.pi))


def sabine_order(size, beta, c=343.0) -> int:
    """Reflection order from Sabine's reverberation time: absorption
    alpha_w = 1 - beta_w^2, RT60 = 0.161 V / sum_w S_w alpha_w, and
    K = clamp(ceil(c RT60 / (Lx + Ly + Lz)), 6, 18)."""
    Lx, Ly, Lz = (float(v) for v in size)
    S = [Ly * Lz, Ly * Lz, Lx * Lz, Lx * Lz, Lx * Ly, Lx * Ly]
    A = sum(s * (1.0 - float(b) ** 2) for s, b in zip(S, beta))
    rt60 = 0.161 * Lx * Ly * Lz / A
    return int(min(18, max(6, math.ceil(c * rt60 / (Lx + Ly + Lz)))))


# ----------------------------------------------------------------- workloads

def config1(seed: int = 1) -> Tuple[List[Scene], Params]:
    """Plain method, tiny: 5x4x3 m, beta 0.9, straight source path
    (1,1,1.5) -> (4,3,1.5) in 1 s, fixed receiver, K = 2, full rate, T = 32."""
    rng = np.random.default_rng(seed)
    size = np.array([5.0, 4.0, 3.0])
    par = Params(fs=16000.0, taps=32, tiers=())
    n_in = 16000
    sc = Scene(size, np.full(6, 0.9), Traj.pwl([0.0, 1.0], [[1, 1, 1.5], [4, 3, 1.5]]),
               Traj.static([2.5, 2.0, 1.2]), np.zeros((1, 3)), noise(rng, n_in),
               n_out_for(size, 2, n_in, par.fs, par.c, par.taps), 2)
    return [sc], par


def config2(seed: int = 2, seconds: float = 4.0) -> Tuple[List[Scene], Params]:
    """Plain method, paper scale: 8x6x3.5 m, beta_w ~ U(0.75, 0.95), 4 s,
    4-knot source path at 0.5-2 m/s, fixed receiver, K = 12, tiers
    16 kHz / 1 kHz / 100 Hz (orders <=2 / 3-6 / >=7), T = 64."""
    rng = np.random.default_rng(seed)
    size = np.array([8.0, 6.0, 3.5])
    par = Params(fs=16000.0, taps=64, tiers=PAPER_TIERS)
    beta = rng.uniform(0.75, 0.95, 6)
    rcv = rng.uniform([0.5, 0.5, 0.5], size - 0.5)
    src = random_pwl(rng, size, 4, seconds, 0.5, 2.0, keep_away=rcv)
    n_in = int(round(seconds * par.fs))
    sc = Scene(size, beta, src, Traj.static(rcv), np.zeros((1, 3)), noise(rng, n_in),
               n_out_for(size, 12, n_in, par.fs, par.c, par.taps), 12)
    return [sc], par


def config3(seed: int = 3, n_scenes: int = 256, max_seconds: float = 8.0) -> Tuple[List[Scene], Params]:
    """Batched forward: independent rooms U(3,10)xU(3,8)xU(2.5,4) m, beta ~
    U(0.7, 0.95), order from Sabine's RT60 (6-18), lengths U(1, max_seconds) s,
    half straight paths and half circles at 0.3-2 m/s, tiers, T = 64."""
    rng = np.random.default_rng(seed)
    par = Params(fs=16000.0, taps=64, tiers=PAPER_TIERS)
    scenes = []
    for s in range(n_scenes):
        size = np.array([rng.uniform(3, 10), rng.uniform(3, 8), rng.uniform(2.5, 4)])
        beta = rng.uniform(0.7, 0.95, 6)
        K = sabine_order(size, beta, par.c)
        secs = rng.uniform(1.0, max_seconds)
        n_in = int(round(secs * par.fs))
        rcv = rng.uniform([0.5, 0.5, 0.5], size - 0.5)
        if s % 2 == 0:
            src = random_pwl(rng, size, 4, secs, 0.3, 2.0, keep_away=rcv)
        else:
            for _ in range(100):
                src = random_circle(rng, size, 0.3, 2.0)
                if abs(src.center[2] - rcv[2]) > 0.3 or np.hypot(src.center[0] - rcv[0], src.center[1] - rcv[1]) > src.radius + 0.5:
                    break
        scenes.append(Scene(size, beta, src, Traj.static(rcv), np.zeros((1, 3)), noise(rng, n_in),
                            n_out_for(size, K, n_in, par.fs, par.c, par.taps), K))
    return scenes, par


def config4(seed: int = 4, n_scenes: int = 32, seconds: float = 2.0, max_order: int = 10) -> Tuple[List[Scene], Params]:
    """Differentiation: 6x5x3 m, 2 s, K = 10, tiers, 8-knot source paths,
    beta_w ~ U(0.75, 0.95)."""
    rng = np.random.default_rng(seed)
    size = np.array([6.0, 5.0, 3.0])
    par = Params(fs=16000.0, taps=64, tiers=PAPER_TIERS)
    scenes = []
    for s in range(n_scenes):
        beta = rng.uniform(0.75, 0.95, 6)
        rcv = rng.uniform([0.5, 0.5, 0.5], size - 0.5)
        src = random_pwl(rng, size, 8, seconds, 0.5, 2.0, keep_away=rcv)
        n_in = int(round(seconds * par.fs))
        scenes.append(Scene(size, beta, src, Traj.static(rcv), np.zeros((1, 3)), noise(rng, n_in),
                            n_out_for(size, max_order, n_in, par.fs, par.c, par.taps), max_order))
    return scenes, par


def config5(seed: int = 5, n_scenes: int = 64, seconds: float = 10.0, max_order: int = 20) -> Tuple[List[Scene], Params]:
    """Large: 12x9x4 m, 48 kHz, 10 s, moving source and receiver (<= 2 m/s),
    8-mic circular array of radius 5 cm, K = 20, tiers at 48 k / 3 k / 300 Hz,
    T = 96."""
    rng = np.random.default_rng(seed)
    size = np.array([12.0, 9.0, 4.0])
    par = Params(fs=48000.0, taps=96, tiers=PAPER_TIERS)
    ang = np.arange(8) * (2 * math.pi / 8)
    mics = np.stack([0.05 * np.cos(ang), 0.05 * np.sin(ang), np.zeros(8)], axis=1)
    scenes = []
    for s in range(n_scenes):
        beta = rng.uniform(0.7, 0.95, 6)
        rcv = random_pwl(rng, size, 6, seconds, 0.1, 2.0, margin=0.6)
        src = random_pwl(rng, size, 6, seconds, 0.1, 2.0, margin=0.6, keep_away=rcv.p[0])
        n_in = int(round(seconds * par.fs))
        scenes.append(Scene(size, beta, src, rcv, mics.copy(), noise(rng, n_in),
                            n_out_for(size, max_order, n_in, par.fs, par.c, par.taps), max_order))
    return scenes, par


def bandlimited_pwl(rng, size, seconds: float, max_speed: float, bandwidth: float = 1.0, knot_rate: float = 8.0,
                    margin: float = 0.5, n_tones: int = 3, z_range: Tuple[float, float] = (1.2, 1.8)) -> Traj:
    """A random band-limited path (Sec. II-C: trajectories are band-limited,
    their spectrum falling with the square of the motion frequency), as a PWL
    path with knot_rate knots per second: per horizontal axis a sum of n_tones
    sinusoids with frequencies U(0.1, bandwidth) Hz and random phases, the height
    a slower sinusoid inside z_range; amplitudes are scaled so the speed between
    knots stays below max_speed and every knot stays margin inside the walls."""
    t = np.arange(0.0, seconds + 1e-12, 1.0 / knot_rate)
    if t[-1] < seconds:
        t = np.append(t, seconds)
    lo = np.array([margin, margin, z_range[0]])
    hi = np.array([size[0] - margin, size[1] - margin, z_range[1]])
    centre = 0.5 * (lo + hi)
    half = 0.5 * (hi - lo)
    shape = np.zeros((t.shape[0], 3))
    for a in range(3):
        f = rng.uniform(0.1, bandwidth if a < 2 else 0.5 * bandwidth, n_tones)
        ph = rng.uniform(0, 2 * math.pi, n_tones)
        w = rng.uniform(0.5, 1.0, n_tones)
        shape[:, a] = np.sum(w[None, :] * np.sin(2 * math.pi * f[None, :] * t[:, None] + ph[None, :]), axis=1)
    shape /= np.maximum(np.abs(shape).max(axis=0), 1e-12)     # each axis in [-1, 1]
    amp = half * rng.uniform(0.3, 0.9, 3)
    p = centre + shape * amp
    v = np.linalg.norm(np.diff(p, axis=0), axis=1) / np.diff(t)
    if v.max() > max_speed:
        p = centre + (p - centre) * (max_speed / v.max())
    return Traj.pwl(t, p)


def e2_scenes(seed: int = 7, n_scenes: int = 12, seconds: float = 2.0, static_every: int = 11,
              spacing: float = 0.15, sector_deg: float = 30.0, max_speed: float = 1.5,
              max_order: Optional[int] = None) -> Tuple[List[Scene], Params, List[str]]:
    """Data generation in the spirit of the paper's dynamic training set (Sec. III):
    random rooms, a two-microphone pair 15 cm apart at a fixed receiver, sources
    that are static in one scene out of every `static_every` (1:10 static to
    dynamic) and otherwise follow band-limited random paths.  Each scene carries a
    label: 'in' when the source starts within +-sector_deg of the pair's
    broadside direction, else 'out' (the D_in / D_out split).  Orders come from
    Sabine's rule unless max_order is given; tiers as in the paper-scale workload."""
    rng = np.random.default_rng(seed)
    par = Params(fs=16000.0, taps=64, tiers=PAPER_TIERS)
    scenes, labels = [], []
    n_in = int(round(seconds * par.fs))
    for s in range(n_scenes):
        size = np.array([rng.uniform(4, 8), rng.uniform(3, 6), rng.uniform(2.5, 3.5)])
        beta = rng.uniform(0.7, 0.95, 6)
        K = sabine_order(size, beta, par.c) if max_order is None else max_order
        phi = rng.uniform(0, math.pi)                       # pair axis, horizontal
        axis = np.array([math.cos(phi), math.sin(phi), 0.0])
        mics = np.stack([-0.5 * spacing * axis, 0.5 * spacing * axis])
        if s % static_every == 0:
            src = Traj.static([rng.uniform(0.5, size[0] - 0.5), rng.uniform(0.5, size[1] - 0.5),
                               rng.uniform(1.2, 1.8)])
        else:
            src = bandlimited_pwl(rng, size, seconds, max_speed)
        # the receiver stays 0.5 m from the path (knots and segment midpoints)
        pts = src.p if src.p.shape[0] == 1 else np.concatenate([src.p, 0.5 * (src.p[1:] + src.p[:-1])])
        for _ in range(1000):
            rcv = np.array([rng.uniform(1.0, size[0] - 1.0), rng.uniform(1.0, size[1] - 1.0), 1.5])
            if np.min(np.linalg.norm(pts - rcv, axis=1)) > 0.5:
                break
        else:
            raise RuntimeError("no receiver position 0.5 m away from the path")
        d0 = src.p[0] - rcv
        broadside = np.array([-axis[1], axis[0], 0.0])
        cosang = abs(np.dot(d0[:2], broadside[:2])) / max(np.linalg.norm(d0[:2]), 1e-12)
        labels.append("in" if cosang >= math.cos(math.radians(sector_deg)) else "out")
        scenes.append(Scene(size, beta, src, Traj.static(rcv), mics, noise(rng, n_in),
                            n_out_for(size, K, n_in, par.fs, par.c, par.taps), K))
    return scenes, par, labels


def small_scene(seed: int = 0, max_order: int = 3, seconds: float = 0.25, fs: float = 16000.0,
                taps: int = 32, tiers=((1, 1), (2, 4), (1 << 20, 16)), n_mics: int = 1,
                moving_rcv: bool = False, circle: bool = False, n_knots: int = 3,
                size=(5.0, 4.0, 3.0)) -> Tuple[Scene, Params]:
    """A small scene the oracle evaluates in seconds, for parity tests."""
    rng = np.random.default_rng(seed)
    size = np.asarray(size, dtype=np.float64)
    par = Params(fs=fs, taps=taps, tiers=tuple(tiers))
    beta = rng.uniform(0.6, 0.95, 6)
    if moving_rcv:
        rcv = random_pwl(rng, size, n_knots, seconds, 0.3, 2.0, margin=0.6)
        anchor = rcv.p[0]
    else:
        anchor = rng.uniform([0.6, 0.6, 0.6], size - 0.6)
        rcv = Traj.static(anchor)
    if circle:
        src = random_circle(rng, size, 0.5, 2.0, r_lo=0.5, r_hi=1.2)
    else:
        src = random_pwl(rng, size, n_knots, seconds, 0.5, 2.0, keep_away=anchor)
    ang = np.arange(n_mics) * (2 * math.pi / max(n_mics, 1))
    mics = np.stack([0.05 * np.cos(ang), 0.05 * np.sin(ang), np.zeros(n_mics)], axis=1) if n_mics > 1 else np.zeros((1, 3))
    n_in = int(round(seconds * fs))
    return Scene(size, beta, src, rcv, mics, noise(rng, n_in),
                 n_out_for(size, max_order, n_in, fs, par.c, taps), max_order), par
