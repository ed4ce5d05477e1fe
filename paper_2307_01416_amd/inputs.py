"""Seeded synthetic workloads for the aperture-block VP transport.

This module only *describes* inputs: phantoms, CT volumes, aperture polygons,
spot maps and robust scenarios.  It contains none of the transport arithmetic
(no stopping powers, ranges, scattering or tallies), so both the HIP product
path and the FP64 oracle can consume the same case objects.

The shapes follow the paper's validation workloads:

* water phantoms with a 30 mm brass block, openings of 1-4 cm, with and
  without a 45 mm WET range shifter 10 mm upstream of the block
  (Methods B, Methods D.1, D.2);
* spots on a 2.5 mm square grid covering the opening plus a 5 mm margin,
  equal intensity, one energy layer (Methods D.2);
* in-air spot sigma falling from 5 mm to 2 mm over 71.3-228.8 MeV
  (Introduction), 97 machine energies in that interval (Methods D.1);
* brain SRS geometry: small, shallow targets, 3 coplanar fields, apertures
  conforming to the target projection plus margin, range shifter
  (Methods D.3, E; Table 1);
* 13 robust scenarios built from range scaling and isocentre shifts along the
  three cardinal axes (Methods E).

Coordinates: mm.  Energies: MeV.  Densities: g/cm^3.  CT arrays are indexed
``hu[k, j, i]`` (x fastest in memory, z slowest).
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Sequence

import numpy as np

E_MIN_MACHINE = 71.3
E_MAX_MACHINE = 228.8
N_MACHINE_ENERGIES = 97

SPOT_DTYPE = np.dtype([
    ("x_mm", np.float32), ("y_mm", np.float32),
    ("energy_mev", np.float32), ("sigma_mm", np.float32),
    ("energy_sigma_mev", np.float32), ("weight", np.float32),
    ("n_histories", np.uint32),
])

GEOM_WATER = 0
GEOM_HU = 1

STRAGGLE = 1
MCS = 2
NUCLEAR = 4
PHYS_ALL = STRAGGLE | MCS | NUCLEAR


# --------------------------------------------------------------------------
# case description
# --------------------------------------------------------------------------
@dataclasses.dataclass
class Geometry:
    kind: int                      # GEOM_WATER or GEOM_HU
    shape: tuple                   # (nx, ny, nz)
    spacing: tuple                 # (dx, dy, dz) mm
    origin: tuple                  # corner of voxel (0,0,0), mm
    hu: Optional[np.ndarray] = None  # int16 [nz, ny, nx] for GEOM_HU

    def __post_init__(self):
        self.spacing = tuple(float(np.float32(x)) for x in self.spacing)
        self.origin = tuple(float(np.float32(x)) for x in self.origin)

    @property
    def nvox(self) -> int:
        nx, ny, nz = self.shape
        return nx * ny * nz


def f32(x) -> float:
    """The value as the C ABI receives it (FP32), so that every consumer of a
    case (library and reference alike) sees the same numbers."""
    return float(np.float32(x))


def f32s(xs) -> tuple:
    return tuple(f32(x) for x in xs)


@dataclasses.dataclass
class Beam:
    """Beam frame: origin at ``iso`` (CT frame), axes given as CT-frame unit
    vectors.  ``ez`` is the beam direction; components sit at negative z."""
    iso: tuple
    ex: tuple
    ey: tuple
    ez: tuple

    def __post_init__(self):
        self.iso, self.ex, self.ey, self.ez = f32s(self.iso), f32s(self.ex), f32s(self.ey), f32s(self.ez)


@dataclasses.dataclass
class Block:
    thickness_mm: float = 30.0
    density_gcc: float = 8.5
    downstream_mm: float = 150.0   # downstream face to the beam-frame origin
    focus_mm: float = 0.0          # walls focused this far upstream of the origin (0: non-divergent)

    def __post_init__(self):
        self.thickness_mm, self.density_gcc, self.downstream_mm, self.focus_mm = f32s(
            (self.thickness_mm, self.density_gcc, self.downstream_mm, self.focus_mm))


@dataclasses.dataclass
class RangeShifter:
    wet_mm: float = 45.0
    diameter_mm: float = 61.0
    downstream_mm: float = 190.0   # downstream face to the beam-frame origin

    def __post_init__(self):
        self.wet_mm, self.diameter_mm, self.downstream_mm = f32s((self.wet_mm, self.diameter_mm, self.downstream_mm))


@dataclasses.dataclass
class Field:
    beam: Beam
    spots: np.ndarray                       # SPOT_DTYPE
    polygon: Optional[np.ndarray] = None    # float32 [n, 2] BEV, mm
    block: Optional[Block] = None           # None: no aperture block at all
    rs: Optional[RangeShifter] = None
    vsad_mm: float = 0.0                    # virtual source upstream of the origin (0: parallel beam)


@dataclasses.dataclass
class Scenario:
    shift_mm: tuple = (0.0, 0.0, 0.0)
    range_scale: float = 1.0

    def __post_init__(self):
        self.shift_mm = f32s(self.shift_mm)
        self.range_scale = f32(self.range_scale)


@dataclasses.dataclass
class Case:
    name: str
    geometry: Geometry
    fields: List[Field]
    scenarios: List[Scenario]
    seed: int = 0
    physics: int = PHYS_ALL
    n_batches: int = 16


# --------------------------------------------------------------------------
# helpers
# --------------------------------------------------------------------------
def machine_energies() -> np.ndarray:
    """97 machine energies 71.3-228.8 MeV, equally spaced (reading: the paper
    gives only the count and the end points)."""
    return np.linspace(E_MIN_MACHINE, E_MAX_MACHINE, N_MACHINE_ENERGIES)


def spot_sigma_mm(energy_mev) -> np.ndarray:
    """In-air spot sigma, linear from 5 mm at 71.3 MeV to 2 mm at 228.8 MeV."""
    e = np.asarray(energy_mev, dtype=np.float64)
    return 5.0 - 3.0 * (e - E_MIN_MACHINE) / (E_MAX_MACHINE - E_MIN_MACHINE)


def make_spots(xy, energy, sigma, n_histories, weight=1.0, energy_sigma=0.0) -> np.ndarray:
    xy = np.asarray(xy, dtype=np.float64).reshape(-1, 2)
    n = xy.shape[0]
    s = np.zeros(n, dtype=SPOT_DTYPE)
    s["x_mm"] = xy[:, 0]
    s["y_mm"] = xy[:, 1]
    s["energy_mev"] = np.broadcast_to(np.asarray(energy, dtype=np.float64), (n,))
    s["sigma_mm"] = np.broadcast_to(np.asarray(sigma, dtype=np.float64), (n,))
    s["energy_sigma_mev"] = energy_sigma
    s["weight"] = np.broadcast_to(np.asarray(weight, dtype=np.float64), (n,))
    s["n_histories"] = np.broadcast_to(np.asarray(n_histories), (n,))
    return s


def beam_along_z(iso) -> Beam:
    """Beam travelling along +z of the CT frame (water-phantom depth axis)."""
    return Beam(iso=tuple(float(v) for v in iso), ex=(1.0, 0.0, 0.0),
                ey=(0.0, 1.0, 0.0), ez=(0.0, 0.0, 1.0))


def beam_coplanar(iso, gantry_deg: float) -> Beam:
    """Coplanar field in the axial (x-y) plane of the CT.  Gantry 0 sends the
    beam along +y; gantry 90 along -x; the beam-frame y axis is CT +z."""
    g = math.radians(gantry_deg)
    a, b = -math.sin(g), math.cos(g)
    # snap tiny values so that axis-aligned gantries give exact unit vectors
    a = 0.0 if abs(a) < 1e-12 else a
    b = 0.0 if abs(b) < 1e-12 else b
    ez = (a, b, 0.0)
    ey = (0.0, 0.0, 1.0)
    ex = (-b, a, 0.0)
    return Beam(iso=tuple(float(v) for v in iso), ex=ex, ey=ey, ez=ez)


def circle_polygon(diameter_mm: float, n: int = 256, center=(0.0, 0.0)) -> np.ndarray:
    """Regular n-gon inscribed in a circle of the given diameter."""
    t = 2.0 * np.pi * (np.arange(n) + 0.5) / n
    r = 0.5 * diameter_mm
    return np.stack([center[0] + r * np.cos(t), center[1] + r * np.sin(t)], 1).astype(np.float32)


def square_grid_in_disk(radius_mm: float, spacing_mm: float = 2.5, center=(0.0, 0.0)) -> np.ndarray:
    m = int(math.floor(radius_mm / spacing_mm)) + 1
    g = np.arange(-m, m + 1) * spacing_mm
    xx, yy = np.meshgrid(g, g, indexing="xy")
    keep = xx ** 2 + yy ** 2 <= radius_mm ** 2 + 1e-9
    return np.stack([xx[keep] + center[0], yy[keep] + center[1]], 1)


def scenarios_13(shift_mm: float = 3.0, range_frac: float = 0.035) -> List[Scenario]:
    """Nominal + 6 isocentre shifts (+-x, +-y, +-z), each at +range and -range
    scaling: 1 + 6*2 = 13 scenarios."""
    out = [Scenario()]
    for axis in range(3):
        for sgn in (+1.0, -1.0):
            sh = [0.0, 0.0, 0.0]
            sh[axis] = sgn * shift_mm
            for rs in (1.0 + range_frac, 1.0 - range_frac):
                out.append(Scenario(shift_mm=tuple(sh), range_scale=rs))
    return out


# --------------------------------------------------------------------------
# configurations
# --------------------------------------------------------------------------
def water_geometry(shape, spacing) -> Geometry:
    return Geometry(kind=GEOM_WATER, shape=tuple(int(v) for v in shape),
                    spacing=tuple(float(v) for v in spacing), origin=(0.0, 0.0, 0.0))


def config1(n_histories: int = 100_000, physics: int = PHYS_ALL, seed: int = 0,
            n_batches: int = 16) -> Case:
    """Water 50x50x100 at 2 mm; one 100 MeV pencil beam, sigma 5 mm, entering
    the z = 0 face at its centre; no aperture, no range shifter."""
    g = water_geometry((50, 50, 100), (2.0, 2.0, 2.0))
    spots = make_spots([(0.0, 0.0)], 100.0, 5.0, n_histories)
    f = Field(beam=beam_along_z((50.0, 50.0, 0.0)), spots=spots)
    return Case("config1", g, [f], [Scenario()], seed=seed, physics=physics, n_batches=n_batches)


CONFIG2_OPENINGS_MM = (10.0, 20.0, 30.0, 40.0)


def config2(opening_mm: float, with_rs: bool, histories_per_case: int = 10_000_000,
            physics: int = PHYS_ALL, seed: int = 0, n_batches: int = 16,
            shape=(200, 200, 300), spacing=(1.0, 1.0, 1.0), n_vertices: int = 256) -> Case:
    """Water phantom behind a 30 mm brass block (density 8.5), downstream face
    50 mm upstream of the water surface; circular opening; one energy layer
    (147.0 MeV without, 161.5 MeV with a 45 mm WET range shifter whose
    downstream face leaves a 10 mm gap to the block)."""
    g = water_geometry(shape, spacing)
    nx, ny, _ = g.shape
    iso = (0.5 * nx * g.spacing[0], 0.5 * ny * g.spacing[1], 0.0)
    energy = 161.5 if with_rs else 147.0
    xy = square_grid_in_disk(0.5 * opening_mm + 5.0, 2.5)
    n_spots = xy.shape[0]
    per_spot = max(1, histories_per_case // n_spots)
    spots = make_spots(xy, energy, spot_sigma_mm(energy), per_spot)
    block = Block(thickness_mm=30.0, density_gcc=8.5, downstream_mm=50.0)
    rs = RangeShifter(wet_mm=45.0, diameter_mm=61.0, downstream_mm=50.0 + 30.0 + 10.0) if with_rs else None
    f = Field(beam=beam_along_z(iso), spots=spots, polygon=circle_polygon(opening_mm, n_vertices),
              block=block, rs=rs)
    name = f"config2_{int(opening_mm)}mm_{'rs' if with_rs else 'nors'}"
    return Case(name, g, [f], [Scenario()], seed=seed, physics=physics, n_batches=n_batches)


def config2_all(**kw) -> List[Case]:
    return [config2(o, rs, **kw) for rs in (False, True) for o in CONFIG2_OPENINGS_MM]


def edge_beamlet_sweep(with_rs: bool, histories: int = 100_000, physics: int = PHYS_ALL,
                       shape=(200, 200, 300), spacing=(1.0, 1.0, 1.0)) -> List[Case]:
    """Single beamlets at the 97 machine energies, aimed at the boundary of a
    10 mm opening (Methods D.1)."""
    out = []
    g = water_geometry(shape, spacing)
    nx, ny, _ = g.shape
    iso = (0.5 * nx * g.spacing[0], 0.5 * ny * g.spacing[1], 0.0)
    for e in machine_energies():
        spots = make_spots([(5.0, 0.0)], e, spot_sigma_mm(e), histories)
        block = Block(30.0, 8.5, 50.0)
        rs = RangeShifter(45.0, 61.0, 90.0) if with_rs else None
        f = Field(beam=beam_along_z(iso), spots=spots, polygon=circle_polygon(10.0, 256),
                  block=block, rs=rs)
        out.append(Case(f"edge_{e:.1f}_{'rs' if with_rs else 'nors'}", g, [f], [Scenario()],
                        physics=physics))
    return out


# --------------------------- synthetic head CT ----------------------------
HEAD_SHAPE = (256, 256, 160)
HEAD_SPACING = (1.0, 1.0, 2.0)
TARGET_VOLUMES_CC = (0.4, 8.0, 43.0)


def sphere_radius_mm(volume_cc: float) -> float:
    return (3.0 * volume_cc * 1000.0 / (4.0 * math.pi)) ** (1.0 / 3.0)


def head_ct(seed: int = 0, shape=HEAD_SHAPE, spacing=HEAD_SPACING) -> Geometry:
    """Seeded synthetic head: ellipsoidal skull shell (7 mm, HU U[1000,1500]),
    brain HU U[20,50], air sinus ellipsoids (HU -1000), air outside, Gaussian
    HU noise sigma 20 on tissue; clamped to [-1024, 3071]."""
    rng = np.random.default_rng(seed)
    nx, ny, nz = shape
    dx, dy, dz = spacing
    x = (np.arange(nx) + 0.5) * dx - 0.5 * nx * dx
    y = (np.arange(ny) + 0.5) * dy - 0.5 * ny * dy
    z = (np.arange(nz) + 0.5) * dz - 0.5 * nz * dz
    Z, Y, X = np.meshgrid(z, y, x, indexing="ij")
    a, b, c = 75.0, 95.0, 70.0          # outer semi-axes (x: left-right, y: ant-post, z: sup-inf)
    t = 7.0
    outer = (X / a) ** 2 + (Y / b) ** 2 + (Z / c) ** 2 <= 1.0
    inner = (X / (a - t)) ** 2 + (Y / (b - t)) ** 2 + (Z / (c - t)) ** 2 <= 1.0
    hu = np.full((nz, ny, nx), -1000.0, dtype=np.float64)
    skull = outer & ~inner
    hu[skull] = rng.uniform(1000.0, 1500.0, size=int(skull.sum()))
    hu[inner] = rng.uniform(20.0, 50.0, size=int(inner.sum()))
    tissue = outer.copy()
    # sinus cavities: anterior-inferior air pockets inside the skull
    for (cx, cy, cz, rx, ry, rz) in ((-18.0, -70.0, -35.0, 12.0, 10.0, 14.0),
                                      (18.0, -70.0, -35.0, 12.0, 10.0, 14.0),
                                      (0.0, -80.0, -10.0, 8.0, 6.0, 8.0)):
        cav = ((X - cx) / rx) ** 2 + ((Y - cy) / ry) ** 2 + ((Z - cz) / rz) ** 2 <= 1.0
        hu[cav] = -1000.0
        tissue &= ~cav
    hu[tissue] += rng.normal(0.0, 20.0, size=int(tissue.sum()))
    hu = np.clip(np.rint(hu), -1024, 3071).astype(np.int16)
    return Geometry(kind=GEOM_HU, shape=(nx, ny, nz), spacing=tuple(spacing),
                    origin=(-0.5 * nx * dx, -0.5 * ny * dy, -0.5 * nz * dz), hu=hu)


def _hu_to_rsp_estimate(hu: np.ndarray) -> np.ndarray:
    """Planning-only water-equivalence estimate used to *choose* spot energies
    (a stand-in for the planner's WET calculation).  Not used by transport."""
    h = hu.astype(np.float64)
    return np.where(h < -900, 0.001, np.where(h < 150, 1.0 + 0.001 * h * 0.6, 1.0 + 0.0005 * h))


def _bragg_kleeman_energy(wet_cm: float) -> float:
    """Textbook Bragg-Kleeman rule R = 0.0022 E^1.77 (cm, MeV), inverted; used
    only to pick layer energies for the synthetic plan."""
    return (max(wet_cm, 1e-6) / 0.0022) ** (1.0 / 1.77)


def _wet_along(geom: Geometry, start, direction, length_mm: float, step=0.5) -> np.ndarray:
    rsp = _hu_to_rsp_estimate(geom.hu)
    nx, ny, nz = geom.shape
    n = int(length_mm / step)
    s = (np.arange(n) + 0.5) * step
    p = np.asarray(start)[None, :] + s[:, None] * np.asarray(direction)[None, :]
    idx = np.floor((p - np.asarray(geom.origin)) / np.asarray(geom.spacing)).astype(int)
    ok = (idx[:, 0] >= 0) & (idx[:, 0] < nx) & (idx[:, 1] >= 0) & (idx[:, 1] < ny) & (idx[:, 2] >= 0) & (idx[:, 2] < nz)
    vals = np.zeros(n)
    vals[ok] = rsp[idx[ok, 2], idx[ok, 1], idx[ok, 0]]
    return np.cumsum(vals) * step


HEAD_TARGET_CENTRES = {0.4: (20.0, 30.0, 10.0), 8.0: (-25.0, 20.0, 20.0), 43.0: (10.0, -15.0, 0.0)}


def config3(target_cc: float = 8.0, histories_per_spot: int = 10_000, physics: int = PHYS_ALL,
            seed: int = 0, gantries=(90.0, 180.0, 270.0), layer_spacing_mm: Optional[float] = None,
            uneven: bool = False, n_vertices: int = 128, geometry: Optional[Geometry] = None,
            scenarios: Optional[Sequence[Scenario]] = None, layer_apertures: bool = False) -> Case:
    """Synthetic head case: one spherical target, 3 coplanar fields, each with
    a brass aperture = BEV projection of the target + 5 mm and a 45 mm WET
    range shifter; spots on a 2.5 mm grid in layers whose cross-section
    follows the target (+5 mm); energies from the 97-energy table.

    layer_apertures: energy-layer-specific apertures (the paper's proposed
    dynamic aperture, Discussion): every energy layer becomes a field of its
    own (same beam, block and range shifter) whose opening is the target's
    cross-section at that layer's depth + 5 mm (n_vertices-gon), i.e. the
    layer's spot disk; fields are ordered gantry by gantry, layer by layer."""
    geom = geometry if geometry is not None else head_ct(seed)
    r = sphere_radius_mm(target_cc)
    centre = HEAD_TARGET_CENTRES.get(target_cc, (0.0, 0.0, 0.0))
    if layer_spacing_mm is None:
        layer_spacing_mm = 2.0 if r < 8 else 3.0
    energies = machine_energies()
    rng = np.random.default_rng(seed + 1000)
    fields = []
    for g in gantries:
        beam = beam_coplanar(centre, g)
        ez = np.asarray(beam.ez)
        start = np.asarray(centre) - 200.0 * ez
        wet = _wet_along(geom, start, ez, 400.0)
        s_axis = (np.arange(wet.size) + 0.5) * 0.5 - 200.0     # beam-frame z of samples
        xy_all, e_all = [], []
        rs_wet_cm = 4.5
        zs = np.arange(-r - 2.0, r + 2.0 + 1e-9, layer_spacing_mm)
        for zl in zs:
            wet_here = float(np.interp(zl, s_axis, wet)) / 10.0 + rs_wet_cm
            e = _bragg_kleeman_energy(wet_here)
            e = float(energies[np.argmin(np.abs(energies - e))])
            rad = math.sqrt(max(r * r - min(zl * zl, r * r), 0.0)) + 5.0
            xy = square_grid_in_disk(rad, 2.5)
            xy_all.append(xy)
            e_all.append(np.full(xy.shape[0], e))
        xy = np.concatenate(xy_all)
        e = np.concatenate(e_all)
        if uneven:
            nh = (histories_per_spot * rng.uniform(0.5, 1.5, size=e.size)).astype(np.uint32)
        else:
            nh = np.full(e.size, histories_per_spot, dtype=np.uint32)
        spots = make_spots(xy, e, spot_sigma_mm(e), 1)
        spots["n_histories"] = nh
        if layer_apertures:
            k0 = 0
            for xy_l in xy_all:
                k1 = k0 + xy_l.shape[0]
                rad = float(np.max(np.hypot(xy_l[:, 0], xy_l[:, 1]))) if xy_l.shape[0] else 5.0
                fields.append(Field(beam=beam, spots=spots[k0:k1].copy(),
                                    polygon=circle_polygon(2.0 * max(rad, 5.0), n_vertices),
                                    block=Block(30.0, 8.5, 150.0), rs=RangeShifter(45.0, 61.0, 190.0)))
                k0 = k1
            continue
        poly = circle_polygon(2.0 * (r + 5.0), n_vertices)
        fields.append(Field(beam=beam, spots=spots, polygon=poly,
                            block=Block(30.0, 8.5, 150.0), rs=RangeShifter(45.0, 61.0, 190.0)))
    scen = list(scenarios) if scenarios is not None else [Scenario()]
    return Case(f"config3_{target_cc}cc", geom, fields, scen, seed=seed, physics=physics)


def config4(target_cc: float = 8.0, histories_per_spot: int = 10_000, **kw) -> Case:
    """13 robust scenarios x 3 fields x all spots (uneven histories) of the
    synthetic head case; per-spot sparse influence matrices."""
    c = config3(target_cc, histories_per_spot, uneven=True, scenarios=scenarios_13(), **kw)
    c.name = f"config4_{target_cc}cc"
    return c


def surrogate_training_entries(n: int, seed: int = 0, polygon: Optional[np.ndarray] = None):
    """Entry states for brass-block traversal samples: energies U[71,229],
    entry points concentrated within +-10 mm of the polygon edges, small
    direction cosines (beam + range-shifter scattering)."""
    rng = np.random.default_rng(seed)
    if polygon is None:
        polygon = circle_polygon(20.0, 256)
    k = rng.integers(0, polygon.shape[0], size=n)
    a = polygon[k].astype(np.float64)
    b = polygon[(k + 1) % polygon.shape[0]].astype(np.float64)
    t = rng.uniform(0.0, 1.0, size=n)
    pt = a + (b - a) * t[:, None]
    c = pt / np.maximum(np.linalg.norm(pt, axis=1, keepdims=True), 1e-9)
    off = rng.uniform(-10.0, 10.0, size=n)
    xy = pt + c * off[:, None]
    ang = rng.normal(0.0, 0.02, size=(n, 2))
    e = rng.uniform(71.0, 229.0, size=n)
    return xy, ang, e


@dataclasses.dataclass
class OptProblem:
    """Influence matrices in CSR (rows (scenario, spot), ascending voxel
    columns, FP32 Gy per unit weight) with target / organ masks, as the
    spot-weight optimiser consumes them."""
    shape: tuple            # (nx, ny, nz), x fastest
    n_scen: int
    n_spots: int
    row_ptr: np.ndarray     # int64 [n_scen * n_spots + 1]
    col: np.ndarray         # int32
    val: np.ndarray         # float32
    roi: np.ndarray         # uint8 [nvox]: bit 0 target, bit 1 organ at risk

    @property
    def nvox(self) -> int:
        return int(np.prod(self.shape))


def opt_problem(seed: int = 0, shape=(40, 36, 20), n_spots: int = 48, n_scen: int = 3,
                empty_rows: int = 2) -> OptProblem:
    """Pencil-beam-like synthetic matrices: each spot covers the voxels of a
    lateral square (half width 2-5 voxels) around its axis along +x, from the
    entrance to a random depth; values fall off laterally and rise towards the
    end of the range; each scenario moves the spot axes by up to 1 voxel.  A
    few rows are empty.  The target is a box in the middle of the grid, the
    organ at risk a slab beside it (a few voxels in both)."""
    rng = np.random.default_rng(seed)
    nx, ny, nz = shape
    jc = rng.uniform(ny * 0.3, ny * 0.7, n_spots)
    kc = rng.uniform(nz * 0.3, nz * 0.7, n_spots)
    hw = rng.integers(2, 6, n_spots)
    depth = rng.integers(nx // 3, nx, n_spots)
    empty = set(rng.choice(n_spots, size=min(empty_rows, n_spots), replace=False).tolist())
    rows_col, rows_val = [], []
    for s in range(n_scen):
        dj, dk = rng.uniform(-1.0, 1.0, 2) if s else (0.0, 0.0)
        for j in range(n_spots):
            if j in empty:
                rows_col.append(np.zeros(0, np.int32))
                rows_val.append(np.zeros(0, np.float32))
                continue
            c0, c1 = jc[j] + dj, kc[j] + dk
            js = np.arange(max(0, int(c0) - hw[j]), min(ny, int(c0) + hw[j] + 1))
            ks = np.arange(max(0, int(c1) - hw[j]), min(nz, int(c1) + hw[j] + 1))
            i = np.arange(0, depth[j])
            K, J, I = np.meshgrid(ks, js, i, indexing="ij")
            lat = np.exp(-((J - c0) ** 2 + (K - c1) ** 2) / (2.0 * (0.5 * hw[j]) ** 2))
            dep = 0.3 + 0.7 * (I / max(1, depth[j] - 1)) ** 4
            v = 1e-3 * lat * dep * rng.uniform(0.9, 1.1, I.shape)
            idx = (K * ny + J) * nx + I
            order = np.argsort(idx.ravel(), kind="stable")
            rows_col.append(idx.ravel()[order].astype(np.int32))
            rows_val.append(v.ravel()[order].astype(np.float32))
    lens = np.array([len(c) for c in rows_col], np.int64)
    row_ptr = np.concatenate([[0], np.cumsum(lens)]).astype(np.int64)
    roi = np.zeros((nz, ny, nx), np.uint8)
    roi[nz // 2 - 3: nz // 2 + 3, ny // 2 - 4: ny // 2 + 4, nx // 2 - 5: nx // 2 + 5] |= 1
    roi[nz // 2 - 3: nz // 2 + 3, ny // 2 + 3: ny // 2 + 8, :] |= 2
    return OptProblem(tuple(shape), n_scen, n_spots, row_ptr, np.concatenate(rows_col).astype(np.int32),
                      np.concatenate(rows_val).astype(np.float32), roi.ravel())


def head_structures(case: Case, target_cc: float = 8.0, oar_radius_mm: float = 8.0, gap_mm: float = 3.0):
    """Structure masks of the synthetic head case for plan optimisation:
    uint8 [nvox], bit 0 = the spherical target, bit 1 = a spherical organ at
    risk of radius oar_radius_mm whose surface lies gap_mm from the target's,
    on the line from the target centre towards the head centre."""
    g = case.geometry
    nx, ny, nz = g.shape
    r = sphere_radius_mm(target_cc)
    c = np.array(HEAD_TARGET_CENTRES.get(target_cc, (0.0, 0.0, 0.0)), np.float64)
    u = -c / max(np.linalg.norm(c), 1e-9) if np.linalg.norm(c) > 0 else np.array([1.0, 0.0, 0.0])
    co = c + u * (r + gap_mm + oar_radius_mm)
    x = g.origin[0] + (np.arange(nx) + 0.5) * g.spacing[0]
    y = g.origin[1] + (np.arange(ny) + 0.5) * g.spacing[1]
    z = g.origin[2] + (np.arange(nz) + 0.5) * g.spacing[2]
    Z, Y, X = np.meshgrid(z, y, x, indexing="ij")
    roi = np.zeros((nz, ny, nx), np.uint8)
    roi[(X - c[0]) ** 2 + (Y - c[1]) ** 2 + (Z - c[2]) ** 2 <= r * r] |= 1
    roi[(X - co[0]) ** 2 + (Y - co[1]) ** 2 + (Z - co[2]) ** 2 <= oar_radius_mm ** 2] |= 2
    return roi.ravel()


def dynamic_spacing_map(shape, roi: np.ndarray, target: int = 1, oar: int = 2, other: int = 4):
    """Voxel -> cell map for dynamic voxel spacing of the influence matrices
    along x (runs of consecutive voxels, never across an x row): target
    voxels (roi bit 0) in runs of `target`, organ-at-risk voxels (bit 1) in
    runs of `oar`, all others in runs of `other`; a run ends where the
    voxels' class changes.  Returns (int32 map [nvox], number of cells)."""
    nx, ny, nz = shape
    cls = np.where((roi & 1) != 0, 0, np.where((roi & 2) != 0, 1, 2)).reshape(nz * ny, nx)
    width = np.array([target, oar, other], np.int64)
    # start of a new cell: first voxel of an x row, a class change, or the
    # run of its class reaching its width
    start = np.zeros((nz * ny, nx), bool)
    start[:, 0] = True
    start[:, 1:] = cls[:, 1:] != cls[:, :-1]
    run = np.zeros(nz * ny, np.int64)
    for i in range(nx):
        run = np.where(start[:, i], 0, run + 1)
        w = width[cls[:, i]]
        hit = (run % w == 0) & ~start[:, i]
        start[:, i] |= hit
    cmap = np.cumsum(start.ravel()) - 1
    return cmap.astype(np.int32), int(cmap[-1]) + 1
