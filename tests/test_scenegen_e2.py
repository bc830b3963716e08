"""The paper-style data front-end (band-limited random paths, a 15 cm mic pair,
1:10 static to dynamic, in/out direction labels): invariants of the generated
inputs, checked on the CPU.  The generator holds no synthesis arithmetic."""
import math

import numpy as np

from paper_2508_03065_amd import scenegen as G


def test_paths_stay_inside_and_below_speed():
    scenes, par, labels = G.e2_scenes(seed=3, n_scenes=22, max_speed=1.5)
    for sc in scenes:
        p = sc.src.p
        assert np.all(p[:, :2] >= 0.5 - 1e-9) and np.all(p[:, :2] <= sc.size[:2] - 0.5 + 1e-9)
        assert np.all(p[:, 2] >= 1.2 - 1e-9) and np.all(p[:, 2] <= 1.8 + 1e-9)
        if p.shape[0] > 1:
            v = np.linalg.norm(np.diff(p, axis=0), axis=1) / np.diff(sc.src.t)
            assert v.max() <= 1.5 + 1e-9
        assert np.min(np.linalg.norm(p - sc.rcv.p[0], axis=1)) > 0.5


def test_static_to_dynamic_ratio_and_pair():
    scenes, _, _ = G.e2_scenes(seed=4, n_scenes=33)
    static = [sc.src.p.shape[0] == 1 for sc in scenes]
    assert sum(static) == 3 and len(static) - sum(static) == 30          # 1:10
    for sc in scenes:
        assert sc.n_mics == 2
        assert abs(np.linalg.norm(sc.mic_offset[1] - sc.mic_offset[0]) - 0.15) < 1e-12
        assert np.allclose(sc.mic_offset[0] + sc.mic_offset[1], 0.0)


def test_direction_labels_follow_the_broadside_sector():
    scenes, _, labels = G.e2_scenes(seed=5, n_scenes=40, sector_deg=30.0)
    assert set(labels) == {"in", "out"}
    for sc, lab in zip(scenes, labels):
        axis = sc.mic_offset[1] - sc.mic_offset[0]
        d = sc.src.p[0] - sc.rcv.p[0]
        # angle between the source direction and the pair axis, folded to [0, 90] deg
        ang = math.degrees(math.atan2(abs(axis[0] * d[1] - axis[1] * d[0]), abs(axis[0] * d[0] + axis[1] * d[1])))
        off_broadside = 90.0 - ang
        assert (lab == "in") == (off_broadside <= 30.0 + 1e-9), (lab, off_broadside)


def test_paths_are_band_limited():
    # the knots sample a sum of tones below 1 Hz at 8 knots per second: the
    # knot sequence's spectrum above 2 Hz holds a negligible share of its energy
    scenes, _, _ = G.e2_scenes(seed=6, n_scenes=11, seconds=8.0)
    for sc in scenes:
        if sc.src.p.shape[0] == 1:
            continue
        p = sc.src.p - sc.src.p.mean(axis=0)
        spec = np.abs(np.fft.rfft(p * np.hanning(p.shape[0])[:, None], axis=0)) ** 2
        f = np.fft.rfftfreq(p.shape[0], d=1.0 / 8.0)
        assert spec[f > 2.0].sum() <= 1e-3 * spec.sum()
