"""The synthetic workloads: seeded meshes, loads, receivers, frequency grids and ROM settings.

  box          rigid-walled air box 1.0 x 0.7 x 0.5 m, 10 x 7 x 5 hex8, 528 pressure DoF,
               unit volume-velocity source, 50 receivers, 481 frequencies 20..500 Hz,
               4 fixed expansion points (80, 200, 320, 440 Hz) x 10 Krylov vectors.
  plate_cavity air box 1.2 x 0.8 x 0.6 m (24 x 16 x 12 hex8) closed on top by a 2 mm clamped
               aluminium plate (24 x 16 x 1 solid hex8), 7,595 DoF, unit normal point force,
               50 receivers, 1000 frequencies 10..400 Hz, greedy expansion points (10 vectors
               per point, relative-residual tolerance 1e-6, at most 24 points).

The paper's fuselage model, its plane-wave load and its measured damping are not available;
these structured models keep the structure of its coupled u-p system (thin damped metal
structure, damped air cavity, coupling on the wetted surface, broadband sweep).
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from .meshes import (FLUID, LOAD_POINT_FORCE, LOAD_VOLUME_VELOCITY, SOLID, Load, Material, Mesh,
                     air_box, fluid_nodes, plate_cavity, solid_nodes)
from .rng import (STREAM_RECEIVERS, STREAM_SOURCE, SplitMix64, stream_seed)

AIR = dict(c=343.0, rho=1.21, eta=0.01)
ALU = dict(E=70e9, nu=0.3, rho=2700.0, eta=0.02)

BOX_ID = 1
PLATE_CAVITY_ID = 2


@dataclass
class Workload:
    name: str
    mesh: Mesh
    loads: list
    receivers: np.ndarray          # node ids carrying a pressure DoF
    freqs_hz: np.ndarray
    rom: dict = field(default_factory=dict)

    @property
    def omegas(self) -> np.ndarray:
        return 2.0 * np.pi * self.freqs_hz


def _air(scale=None):
    a = dict(AIR)
    if scale:
        a.update(scale)
    return Material(kind=FLUID, rho=a["rho"], eta=a["eta"], c=a["c"])


def box(cells=(10, 7, 5), dims=(1.0, 0.7, 0.5), n_receivers=50) -> Workload:
    mesh = air_box(*dims, *cells, _air())
    fn = fluid_nodes(mesh)
    src = int(SplitMix64(stream_seed(BOX_ID, STREAM_SOURCE)).sample(fn, 1)[0])
    rest = fn[fn != src]
    rec = np.sort(SplitMix64(stream_seed(BOX_ID, STREAM_RECEIVERS)).sample(rest, n_receivers))
    loads = [Load(kind=LOAD_VOLUME_VELOCITY, node=src, value=1.0 + 0.0j)]
    freqs = np.arange(20.0, 500.0 + 0.5, 1.0)
    rom = dict(mode="fixed", shifts_hz=np.array([80.0, 200.0, 320.0, 440.0]), blocks=10)
    return Workload("box", mesh, loads, rec, freqs, rom)


def plate_cavity_workload(cells=(24, 16, 12), dims=(1.2, 0.8, 0.6), t=0.002,
                          n_receivers=50, n_freq=1000, band=(10.0, 400.0)) -> Workload:
    plate = Material(kind=SOLID, rho=ALU["rho"], eta=ALU["eta"], E=ALU["E"], nu=ALU["nu"])
    mesh = plate_cavity(*dims, *cells, t, _air(), plate)
    top = mesh.meta["top_nodes"]
    free_top = np.setdiff1d(top, mesh.clamped)
    src = int(SplitMix64(stream_seed(PLATE_CAVITY_ID, STREAM_SOURCE)).sample(free_top, 1)[0])
    fn = fluid_nodes(mesh)
    rec = np.sort(SplitMix64(stream_seed(PLATE_CAVITY_ID, STREAM_RECEIVERS)).sample(fn, n_receivers))
    loads = [Load(kind=LOAD_POINT_FORCE, node=src, dir=2, value=1.0 + 0.0j)]
    freqs = np.linspace(band[0], band[1], n_freq)
    rom = dict(mode="greedy", band_hz=band, n_cand=256, blocks=10, tol=1e-6, max_shifts=24)
    return Workload("plate_cavity", mesh, loads, rec, freqs, rom)


def small_plate_cavity() -> Workload:
    """A coarse plate-cavity (6 x 4 x 3 cells, 8 receivers) for quick parity cases."""
    w = plate_cavity_workload(cells=(6, 4, 3), n_receivers=8, n_freq=64)
    w.name = "plate_cavity_small"
    w.rom = dict(mode="greedy", band_hz=(10.0, 400.0), n_cand=64, blocks=4, tol=1e-6,
                 max_shifts=12)
    return w


__all__ = ["Workload", "box", "plate_cavity_workload", "small_plate_cavity", "fluid_nodes",
           "solid_nodes"]
