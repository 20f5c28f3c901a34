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
from .rng import (STREAM_ORDERS, STREAM_RECEIVERS, STREAM_SOURCE, STREAM_SPLIT, STREAM_VARIANT, SplitMix64,
                  stream_seed)

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


BATCHED_ID = 4


def batched_variants(n_rom=256, q_range=(40, 400), n_freq=4000, n_loads=16, plate_cells=(24, 16, 12),
                     box_cells=(10, 7, 5)):
    """Seeded variants for the batched sweep: model m is a box variant (m even: rho0 and eta_f
    scaled by U[0.8, 1.2)) or a plate-cavity variant (m odd: E, rho_s, rho0 and eta_s scaled by
    U[0.8, 1.2)), each with n_loads seeded unit loads (volume-velocity sources in the box, normal
    point forces on the plate), a target reduced order q = q_lo + floor((q_hi - q_lo + 1) u), the
    expansion points at the midpoints of 4 sub-bands of [f_lo, 4 f_hi] with ceil(q / (4 L))
    blocks each (the model is then truncated to its first q columns), and n_freq frequencies over
    the model's band.
    Returns a list of (Workload, q_target)."""
    rv = SplitMix64(stream_seed(BATCHED_ID, STREAM_VARIANT))
    rq = SplitMix64(stream_seed(BATCHED_ID, STREAM_ORDERS))
    out = []
    for m in range(n_rom):
        u = rv.uniforms(4)
        s = 0.8 + 0.4 * u
        q = q_range[0] + min(int((q_range[1] - q_range[0] + 1) * rq.uniform()), q_range[1] - q_range[0])
        rl = SplitMix64(stream_seed(BATCHED_ID, STREAM_SOURCE) + 7919 * m)
        if m % 2 == 0:
            air = Material(kind=FLUID, rho=AIR["rho"] * s[0], eta=AIR["eta"] * s[1], c=AIR["c"])
            mesh = air_box(1.0, 0.7, 0.5, *box_cells, air)
            fn = fluid_nodes(mesh)
            src = rl.sample(fn, n_loads)
            loads = [Load(kind=LOAD_VOLUME_VELOCITY, node=int(v), value=1.0 + 0.0j) for v in src]
            rest = np.setdiff1d(fn, src)
            rec = np.sort(rl.sample(rest, 50))
            band = (20.0, 500.0)
        else:
            plate = Material(kind=SOLID, rho=ALU["rho"] * s[1], eta=ALU["eta"] * s[3], E=ALU["E"] * s[0],
                             nu=ALU["nu"])
            air = Material(kind=FLUID, rho=AIR["rho"] * s[2], eta=AIR["eta"], c=AIR["c"])
            mesh = plate_cavity(1.2, 0.8, 0.6, *plate_cells, 0.002, air, plate)
            free_top = np.setdiff1d(mesh.meta["top_nodes"], mesh.clamped)
            src = rl.sample(free_top, n_loads)
            loads = [Load(kind=LOAD_POINT_FORCE, node=int(v), dir=2, value=1.0 + 0.0j) for v in src]
            rec = np.sort(rl.sample(fluid_nodes(mesh), 50))
            band = (10.0, 400.0)
        # expansion points: midpoints of 4 sub-bands of [f_lo, 4 f_hi]; inside the swept band alone
        # the Krylov space of these small models saturates (columns deflate at the 1e-10 ratio)
        # below the orders up to 400 that the batch asks for
        edges = np.linspace(band[0], 4.0 * band[1], 5)
        shifts = 0.5 * (edges[:-1] + edges[1:])
        blocks = int(np.ceil(q / (n_loads * len(shifts))))
        w = Workload(f"variant{m}", mesh, loads, rec, np.linspace(band[0], band[1], n_freq),
                     dict(mode="fixed", shifts_hz=shifts, blocks=blocks, q_target=q))
        out.append((w, q))
    return out


FUSELAGE_ID = 3
LEARNED_ID = 5


def _skin_loads(mesh, n_loads, seed_base):
    """Unit-amplitude skin pressures with independent uniform random phase per outer-skin node."""
    from .meshes import LOAD_SKIN_PRESSURE
    faces = mesh.meta["skin_faces"]
    nodes = np.unique(faces.ravel())
    loads = []
    for l in range(n_loads):
        r = SplitMix64(seed_base + l)
        amp = np.zeros(mesh.n_nodes, complex)
        amp[nodes] = np.exp(2j * np.pi * r.uniforms(len(nodes)))
        loads.append(Load(kind=LOAD_SKIN_PRESSURE, faces=faces, amp=amp))
    return loads


def fuselage_workload(n_core=36, n_ring=18, h_z=0.04, n_loads=16, n_freq=2000, length=4.0, skin_t=0.002,
                      frame_z=(0.4, 1.2, 2.0, 2.8, 3.6), name="fuselage") -> Workload:
    """Cylinder R = 1.4 m, L = 4 m, 2 mm aluminium skin hex layer, 5 frames 60 mm deep (2 mm thick),
    interior air (O-grid); ~6e5 DoF at the default resolution. 16 random-phase skin pressures,
    50 receivers, 2000 frequencies 20..300 Hz, greedy with 4 blocks per expansion point."""
    from .fuselage import fuselage
    plate = Material(kind=SOLID, rho=ALU["rho"], eta=ALU["eta"], E=ALU["E"], nu=ALU["nu"])
    mesh = fuselage(length=length, skin_t=skin_t, frame_z=frame_z, n_core=n_core, n_ring=n_ring, h_z=h_z,
                    air=_air(), metal=plate)
    loads = _skin_loads(mesh, n_loads, stream_seed(FUSELAGE_ID, 3) * 100)
    fn = fluid_nodes(mesh)
    rec = np.sort(SplitMix64(stream_seed(FUSELAGE_ID, STREAM_RECEIVERS)).sample(fn, 50))
    rom = dict(mode="greedy", band_hz=(20.0, 300.0), n_cand=256, blocks=4, tol=1e-6, max_shifts=32)
    return Workload(name, mesh, loads, rec, np.linspace(20.0, 300.0, n_freq), rom)


def fuselage_variants(n_var=64, n_loads=16, n_core=6, n_ring=3, h_z=0.25):
    """Seeded fuselage variants for the learned proposer: length ~ U[2, 5] m, frame pitch
    ~ U[0.4, 0.8] m (frames at pitch (i + 1/2)), skin ~ U[1.5, 3] mm; coarse mesh; n_loads
    random-phase skin pressures; greedy on 256 candidates 20..300 Hz with 2 blocks per point to
    a relative residual of 1e-3: with ||A|| ||x|| / ||f|| ~ 4e7 on these thin-skin models (after
    Jacobi scaling) the residual relative to ||f|| stalls near 1e-4 once new Krylov columns fall
    under the 1e-10 deflation ratio, so 1e-6 is out of reach.
    Returns a list of (Workload, geometry features) and the seeded train/test split (48 / 16)."""
    from .fuselage import fuselage
    rv = SplitMix64(stream_seed(LEARNED_ID, STREAM_VARIANT))
    out = []
    for m in range(n_var):
        u = rv.uniforms(3)
        length = 2.0 + 3.0 * u[0]
        pitch = 0.4 + 0.4 * u[1]
        skin = 1.5e-3 + 1.5e-3 * u[2]
        frames = [pitch * (i + 0.5) for i in range(int(length / pitch + 0.5)) if pitch * (i + 0.5) < length - 0.05]
        plate = Material(kind=SOLID, rho=ALU["rho"], eta=ALU["eta"], E=ALU["E"], nu=ALU["nu"])
        mesh = fuselage(length=length, skin_t=skin, frame_z=frames, n_core=n_core, n_ring=n_ring, h_z=h_z,
                        air=_air(), metal=plate)
        loads = _skin_loads(mesh, n_loads, stream_seed(LEARNED_ID, 3) * 1000 + 100 * m)
        rec = np.sort(SplitMix64(stream_seed(LEARNED_ID, STREAM_RECEIVERS) + m).sample(fluid_nodes(mesh), 50))
        rom = dict(mode="greedy", band_hz=(20.0, 300.0), n_cand=256, blocks=2, tol=1e-3, max_shifts=40)
        geom = np.array([(length - 3.5) / 1.5, (pitch - 0.6) / 0.2, (skin - 2.25e-3) / 0.75e-3])
        out.append((Workload(f"fuselage_variant{m}", mesh, loads, rec, np.linspace(20.0, 300.0, 256), rom), geom))
    perm = SplitMix64(stream_seed(LEARNED_ID, STREAM_SPLIT)).sample(np.arange(n_var), n_var)
    n_train = (3 * n_var) // 4
    return out, np.sort(perm[:n_train]), np.sort(perm[n_train:])


__all__ = ["Workload", "box", "plate_cavity_workload", "small_plate_cavity", "fluid_nodes",
           "solid_nodes", "batched_variants", "fuselage_workload", "fuselage_variants"]
