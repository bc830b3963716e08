"""Tiering error of the oracle against its own full-rate mode (Sec. II-C-3:
high-order images sampled sparsely and interpolated to the audio rate).  The
paper states no SNR for this; these are the values measured here, kept as
lower bounds so a regression in the tier-emulating path shows up.

  * paper-scale room (config 2 geometry, K = 12, 4-knot path), tiers 16 kHz /
    1 kHz / 100 Hz: 43 dB on 0.25 s (46 dB on 0.5 s).  The path's kinks limit it.
  * a 1 kHz sine from a source on a slow circle (0.5 m/s), K = 4, 0.5 s: 225 dB
    with the three tiers, 127 dB with a 16 kHz / 25 Hz split, 85 dB with the
    paper's own 16 kHz / 5 Hz split (ratio 3200)."""
import dataclasses

import numpy as np

from oracle import oracle as O
from paper_2508_03065_amd import scenegen as G


def snr(y, ref):
    return 10 * np.log10(np.sum(ref ** 2) / np.sum((y - ref) ** 2))


def test_paper_tiers_on_paper_scale_room():
    (sc,), par = G.config2(seconds=0.25)
    full = O.forward(sc, dataclasses.replace(par, tiers=()))
    tiered = O.forward(sc, par)
    assert snr(tiered, full) >= 40.0


def test_sine_on_slow_curve_with_sparse_tiers():
    fs, n_in = 16000.0, 8000
    x = np.sin(2 * np.pi * 1000.0 * np.arange(n_in) / fs).astype(np.float32)
    size = np.array([8.0, 6.0, 3.5])
    src = G.Traj.circle(center=[5.0, 3.0, 1.5], radius=1.5, speed=0.5, phase0=np.pi)
    par = G.Params(fs=fs, taps=64, tiers=())
    sc = G.Scene(size, np.full(6, 0.85), src, G.Traj.static([2.0, 3.0, 1.5]), np.zeros((1, 3)), x,
                 G.n_out_for(size, 4, n_in, fs, par.c, par.taps), 4)
    full = O.forward(sc, par)
    for tiers, bound in ((G.PAPER_TIERS, 150.0), (((2, 1), (1 << 20, 640)), 100.0),
                         (((2, 1), (1 << 20, 3200)), 70.0)):
        assert snr(O.forward(sc, dataclasses.replace(par, tiers=tiers)), full) >= bound, tiers
