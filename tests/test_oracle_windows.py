"""Pins of the oracle's local reduced models on frequency windows (CPU)."""
import numpy as np

import workloads as W
from oracle import assembly, greedy, rom, solve, windows


def _small():
    w = W.small_plate_cavity()
    return w, assembly.assemble(w.mesh, w.loads, w.receivers)


def test_windows_partition_the_band_and_converge():
    """Capped at four expansion points the whole band does not converge; bisection gives
    contiguous windows that share their edge candidates, cover the band, and each converges
    (checked against full solves at the window's own candidates)."""
    w, s = _small()
    rp = w.rom
    g = greedy.greedy(s, rp["band_hz"], rp["n_cand"], rp["blocks"], rp["tol"], 4)
    assert g["maxres"][-1] > rp["tol"]
    wins = windows.local_roms(s, rp["band_hz"], rp["n_cand"], rp["blocks"], rp["tol"], 4, 4)
    assert [(x["i0"], x["i1"]) for x in wins] == [(0, 31), (31, 47), (47, 55), (55, 63)]
    assert wins[0]["i0"] == 0 and wins[-1]["i1"] == rp["n_cand"] - 1
    for a, b in zip(wins[:-1], wins[1:]):
        assert a["i1"] == b["i0"]
    cand = np.linspace(*rp["band_hz"], rp["n_cand"])
    for win in wins:
        assert win["greedy"]["maxres"][-1] <= rp["tol"]
        assert len(win["greedy"]["shift_idx"]) <= 4
        om = 2 * np.pi * cand[win["i0"]:win["i1"] + 1:3]
        err = rom.relative_error(rom.sweep(win["greedy"]["rom"], om), solve.full_frf(s, om))
        assert err.max() < 1e-4


def test_windows_stop_at_the_minimum_size():
    """A window is split only while both halves keep at least min_cand candidates; windows left
    unconverged are exactly the ones at the minimum size."""
    w, s = _small()
    rp = w.rom
    wins = windows.local_roms(s, rp["band_hz"], rp["n_cand"], rp["blocks"], rp["tol"], 1, 4)
    for x in wins:
        k = x["i1"] - x["i0"] + 1
        assert k >= 4
        assert x["greedy"]["maxres"][-1] <= rp["tol"] or k < 2 * 4 - 1


def test_one_window_when_the_cap_suffices():
    w, s = _small()
    rp = w.rom
    g = greedy.greedy(s, rp["band_hz"], rp["n_cand"], rp["blocks"], rp["tol"], rp["max_shifts"])
    wins = windows.local_roms(s, rp["band_hz"], rp["n_cand"], rp["blocks"], rp["tol"], rp["max_shifts"], 4)
    assert len(wins) == 1
    assert list(wins[0]["greedy"]["shift_idx"]) == list(g["shift_idx"])
    om = w.omegas
    Yw, owner = windows.sweep(wins, om)
    assert np.all(owner == 0)
    assert np.allclose(Yw, rom.sweep(g["rom"], om), rtol=0, atol=0)


def test_stitched_sweep_routes_each_frequency_to_its_window():
    w, s = _small()
    rp = w.rom
    wins = windows.local_roms(s, rp["band_hz"], rp["n_cand"], rp["blocks"], rp["tol"], 2, 4)
    assert len(wins) > 4
    om = 2 * np.pi * np.linspace(rp["band_hz"][0], rp["band_hz"][1] + 5.0, 97)
    Y, owner = windows.sweep(wins, om)
    f = om / (2 * np.pi)
    for k in range(len(om)):
        win = wins[owner[k]]
        assert f[k] <= win["hi_hz"] or owner[k] == len(wins) - 1
        assert owner[k] == 0 or f[k] > wins[owner[k] - 1]["hi_hz"]
        assert np.array_equal(Y[k], rom.sweep(win["greedy"]["rom"], om[k:k + 1])[0])
