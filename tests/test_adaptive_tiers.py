"""Bandwidth-adaptive decimation per image (Sec. II-C-1/2: a far image's delay
carries the motion's bandwidth, a close image needs a higher rate, faint images
can be sampled sparsely), oracle side.  Image m's delay-error budget is
tier_tol * max(d_m, 0.1) / beta_m samples (d_m the gap between its box over the
path and the mic box, beta_m its reflection product).  Pins, on smooth paths
where the derivative bound is rigorous:
  * the tier-emulated delay of every image stays within its budget of the exact
    delay (the rule's purpose), on a circle and on a straight pass (away from
    where the pass starts and stops: kinks, which no derivative bound covers);
  * near-field detection: the direct image's decimation falls as the receiver
    comes closer to the path, and stays above that of no farther image;
  * a static scene takes the largest decimation for every image;
  * a straight pass with the closest approach d, speed u: the decimation the
    rule gives is the largest ladder value R with R^3 D3 / 24 <= tol for the
    closed-form D3 = (2/sqrt 3) u^3 / (d^2 c fs^2) / (1 - u/c)^3."""
import dataclasses
import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_2508_03065_amd import scenegen as G


def scene(src, rcv_pos, seconds=1.0, K=3, fs=16000.0, size=(8.0, 6.0, 3.5)):
    size = np.asarray(size)
    n_in = int(seconds * fs)
    par = G.Params(fs=fs, taps=32, tiers=(), tier_mode=1, tier_tol=1e-3, tier_rmax=1024)
    sc = G.Scene(size, np.full(6, 0.8), src, G.Traj.static(rcv_pos), np.zeros((1, 3)),
                 np.zeros(n_in, np.float32), G.n_out_for(size, K, n_in, fs, par.c, par.taps), K)
    return sc, par


def images(K):
    out = []
    for mx in range(-K, K + 1):
        for my in range(-K, K + 1):
            for mz in range(-K, K + 1):
                if abs(mx) + abs(my) + abs(mz) <= K:
                    out.append((mx, my, mz))
    return out


def beta_of(sc, m):
    """Reflection product of image m: |m| hits alternating between an axis's walls."""
    b = 1.0
    for a in range(3):
        k = abs(m[a])
        far = (k + 1) // 2 if m[a] >= 0 else k // 2
        b *= sc.beta[2 * a] ** (k - far) * sc.beta[2 * a + 1] ** far
    return b


def gap(sc, m):
    """Distance between image m's box over the path and the mic box (a circle's box
    is its square in its plane)."""
    if sc.src.kind == G.CIRCLE:
        c, r = np.asarray(sc.src.center), sc.src.radius
        lo, hi = c - [r, r, 0.0], c + [r, r, 0.0]
    else:
        lo, hi = sc.src.p.min(axis=0), sc.src.p.max(axis=0)
    mic = sc.rcv.p[0] + sc.mic_offset[0]
    d2 = 0.0
    for a in range(3):
        L = sc.size[a]
        if m[a] % 2 == 0:
            ilo, ihi = m[a] * L + lo[a], m[a] * L + hi[a]
        else:
            ilo, ihi = (m[a] + 1) * L - hi[a], (m[a] + 1) * L - lo[a]
        d2 += max(0.0, ilo - mic[a], mic[a] - ihi) ** 2
    return math.sqrt(d2)


@pytest.mark.parametrize("path", ["circle", "line"])
def test_emulated_delays_within_tolerance(path):
    if path == "circle":
        src = G.Traj.circle(center=[4.0, 3.0, 1.5], radius=1.0, speed=1.5, phase0=0.3)
    else:
        src = G.Traj.pwl([0.0, 1.0], [[1.0, 2.0, 1.5], [7.0, 2.5, 1.5]])     # one piece: no knot inside
    sc, par = scene(src, [4.0, 3.6, 1.2])
    full = dataclasses.replace(par, tier_mode=0, tiers=())
    # the path rests before t = 0 and after its last knot: kinks the bound does not
    # cover, so the outputs checked keep three largest decimations plus the largest
    # delay away from them
    lo = 3 * par.tier_rmax + 2000
    hi = int(par.fs) - 3 * par.tier_rmax
    idx = np.sort(np.random.default_rng(1).choice(hi - lo, 1500, replace=False)) + lo
    t_ad = O.delays(sc, par, 0, idx) * par.fs
    t_ex = O.delays(sc, full, 0, idx) * par.fs
    err = np.max(np.abs(t_ad - t_ex), axis=1)
    ims = images(sc.max_order)
    R = np.array([O.image_decim(sc, par, m) for m in ims])
    assert R.max() >= 4                                  # decimation happens
    budget = np.array([par.tier_tol * max(gap(sc, m), 0.1) / beta_of(sc, m) for m in ims])
    assert np.all(err <= budget), (np.max(err / budget), R[np.argmax(err / budget)])
    assert np.any(err > 0.05 * budget)                   # and the bound is not idle


def test_near_field_lowers_the_direct_image_rate():
    src = G.Traj.circle(center=[4.0, 3.0, 1.5], radius=1.0, speed=1.5, phase0=0.0)
    Rd = []
    for gap in (2.0, 1.0, 0.5, 0.2):
        sc, par = scene(src, [5.0 + gap, 3.0, 1.5])
        R = {m: O.image_decim(sc, par, m) for m in images(2)}
        Rd.append(R[(0, 0, 0)])
        assert all(R[(0, 0, 0)] <= r for r in R.values())
    assert Rd == sorted(Rd, reverse=True) and Rd[0] > Rd[-1]


def test_static_scene_takes_largest_decimation():
    sc, par = scene(G.Traj.static([3.0, 2.0, 1.4]), [5.0, 4.0, 1.2])
    par = dataclasses.replace(par, tier_rmax=500)
    assert {O.image_decim(sc, par, m) for m in images(2)} == {256}


def test_straight_pass_closed_form():
    u, d = 2.0, 0.5
    src = G.Traj.pwl([0.0, 2.0], [[2.0, 3.0 - d, 1.5], [2.0 + 2 * u, 3.0 - d, 1.5]])
    sc, par = scene(src, [4.0, 3.0, 1.5], seconds=2.0, K=0)
    c, fs = par.c, par.fs
    d3 = (2 / math.sqrt(3)) * u ** 3 / (d * d * c * fs * fs) / (1 - u / c) ** 3
    want = 1
    r = 4
    while r <= par.tier_rmax:
        if r ** 3 * d3 <= 24 * par.tier_tol * d:          # the direct image: beta 1, gap d
            want = r
        r *= 2
    assert O.image_decim(sc, par, (0, 0, 0)) == want
