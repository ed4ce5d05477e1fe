"""Thin ctypes binding of libvpmc.so (include/vpmc.h).

Argument marshalling only: every step of the transport runs in the HIP
library.  PyTorch supplies device memory and the stream.  There is no CPU
fallback: if the library is missing, import-time loading raises.
"""
from __future__ import annotations

import ctypes as C
import os
import re
from typing import List, Optional, Sequence

import numpy as np

from . import inputs as I

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libvpmc.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "vpmc.h")

VPMC_OK = 0
ERRORS = {-1: "VPMC_E_ARG", -2: "VPMC_E_STATE", -3: "VPMC_E_POLYGON", -4: "VPMC_E_OOM",
          -5: "VPMC_E_DEVICE", -6: "VPMC_E_RANGE", -7: "VPMC_E_ABORTED"}
E_ARG, E_STATE, E_POLYGON, E_OOM, E_DEVICE, E_RANGE, E_ABORTED = -1, -2, -3, -4, -5, -6, -7
STRAGGLE, MCS, NUCLEAR, PHYS_ALL = 1, 2, 4, 7
GEOM_WATER, GEOM_HU = 0, 1
OUT_DOSE, OUT_CSR = 0, 1
DEVICE_PTRS = 1
GRAPH = 2
SURROGATE = 4
LET = 8
OPT_REUSE = 16
NLEDGER = 6


class VpmcError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{ERRORS.get(code, code)}: {msg}")
        self.code = code


class vpmc_beam(C.Structure):
    _fields_ = [("iso_mm", C.c_float * 3), ("ex", C.c_float * 3), ("ey", C.c_float * 3),
                ("ez", C.c_float * 3)]


class vpmc_block(C.Structure):
    _fields_ = [("thickness_mm", C.c_float), ("density_gcc", C.c_float), ("downstream_mm", C.c_float)]


class vpmc_rs(C.Structure):
    _fields_ = [("wet_mm", C.c_float), ("diameter_mm", C.c_float), ("downstream_mm", C.c_float)]


class vpmc_spot(C.Structure):
    _fields_ = [("x_mm", C.c_float), ("y_mm", C.c_float), ("energy_mev", C.c_float),
                ("sigma_mm", C.c_float), ("energy_sigma_mev", C.c_float), ("weight", C.c_float),
                ("n_histories", C.c_uint32)]


class vpmc_scenario(C.Structure):
    _fields_ = [("shift_mm", C.c_float * 3), ("range_scale", C.c_float)]


class vpmc_opts(C.Structure):
    _fields_ = [("seed", C.c_uint64), ("physics", C.c_uint), ("n_batches", C.c_int),
                ("output", C.c_int), ("fixed_point_bits", C.c_int), ("flags", C.c_uint),
                ("hip_stream", C.c_void_p), ("max_device_bytes", C.c_size_t),
                ("block_threads", C.c_int), ("grid_blocks", C.c_int), ("hist_per_lane", C.c_int),
                ("max_slots", C.c_int), ("queue_cap", C.c_uint64)]


class vpmc_opt_params(C.Structure):
    _fields_ = [("d_presc", C.c_double), ("w_target", C.c_double), ("d_max", C.c_double),
                ("w_oar", C.c_double), ("iters", C.c_int), ("n_power", C.c_int), ("row_stride", C.c_int),
                ("row_offset", C.c_int), ("flags", C.c_uint), ("hip_stream", C.c_void_p)]


class vpmc_stats(C.Structure):
    _fields_ = [("transport_ms", C.c_double), ("total_ms", C.c_double), ("histories", C.c_uint64),
                ("steps", C.c_uint64), ("launches", C.c_uint64), ("deferred", C.c_uint64)]


assert C.sizeof(vpmc_spot) == 28
_lib = None


def load() -> C.CDLL:
    """Load the built library; raise if it is missing (no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"libvpmc.so not built ({LIB_PATH}); run __graft_entry__.build()")
    L = C.CDLL(LIB_PATH)
    vp, i, u, f64p = C.c_void_p, C.c_int, C.c_uint, C.POINTER(C.c_double)
    sig = {
        "vpmc_create": (i, [C.POINTER(vp), i]),
        "vpmc_destroy": (None, [vp]),
        "vpmc_last_error": (C.c_char_p, [vp]),
        "vpmc_version": (i, []),
        "vpmc_load_geometry": (i, [vp, i, vp, i, i, i, vp, vp, u]),
        "vpmc_set_aperture": (i, [vp, i, vp, vp, i, vp, vp]),
        "vpmc_set_divergence": (i, [vp, i, C.c_float, C.c_float]),
        "vpmc_run_spots": (i, [vp, i, vp, i, vp, i, vp, vp, vp, vp, vp]),
        "vpmc_run_spots_noalloc": (i, [vp, i, vp, i, vp, i, vp, vp, vp, vp]),
        "vpmc_copy_csr": (i, [vp, vp, vp, vp]),
        "vpmc_last_tally": (i, [vp, i, vp, C.POINTER(C.c_int), u]),
        "vpmc_last_let": (i, [vp, i, vp, C.POINTER(C.c_int), u]),
        "vpmc_table_host": (i, [i, i, vp, i]),
        "vpmc_last_stats": (i, [vp, vp]),
        "vpmc_run_batched": (i, [vp, vp, vp, vp, i, vp, i, vp, vp, vp, vp]),
        "vpmc_autotune": (i, [vp, i, vp, i, vp, vp, C.c_uint64, vp]),
        "vpmc_surrogate_param_count": (i, []),
        "vpmc_surrogate_sample": (i, [vp, i, vp, i, C.c_uint64, u, vp, vp, vp]),
        "vpmc_surrogate_set_weights": (i, [vp, vp, i]),
        "vpmc_surrogate_config": (i, [vp, C.c_float, C.c_float, C.c_float]),
        "vpmc_surrogate_get_weights": (i, [vp, vp, i]),
        "vpmc_surrogate_load": (i, [vp, C.c_char_p]),
        "vpmc_surrogate_save": (i, [vp, C.c_char_p]),
        "vpmc_surrogate_forward": (i, [vp, vp, i, vp]),
        "vpmc_surrogate_loss_grad": (i, [vp, vp, vp, vp, i, vp, C.POINTER(C.c_double)]),
        "vpmc_surrogate_train": (i, [vp, vp, vp, vp, i, i, i, C.c_float, C.c_uint64, vp]),
        "vpmc_atomic_rate": (i, [vp, i, i, i, C.c_uint64, f64p]),
        "vpmc_optimize": (i, [vp, vp, vp, vp, i, i, i, vp, vp, vp, vp, f64p, vp]),
        "vpmc_csr_cells": (i, [vp, vp, i, vp, vp, i, vp, i, vp, vp, vp, vp, u]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(L, name)
        fn.restype = res
        fn.argtypes = args
    _lib = L
    return L


def header_functions() -> List[str]:
    """Function names declared in include/vpmc.h."""
    txt = open(HEADER).read()
    return sorted(set(re.findall(r"\b(vpmc_[a-z_]+)\s*\(", txt)))


def _check(rc: int, ctx=None):
    if rc != VPMC_OK:
        msg = load().vpmc_last_error(ctx)
        raise VpmcError(rc, msg.decode() if msg else "")


def _f3(v):
    return (C.c_float * 3)(*[float(x) for x in v])


def _ptr(x):
    """Pointer of a numpy array or a torch tensor (host or device), or None."""
    if x is None:
        return None
    if isinstance(x, np.ndarray):
        return x.ctypes.data_as(C.c_void_p)
    return C.c_void_p(x.data_ptr())


# --------------------------------------------------------------- C-ABI mirror
def vpmc_create(device: int = 0) -> C.c_void_p:
    ctx = C.c_void_p()
    _check(load().vpmc_create(C.byref(ctx), device))
    return ctx


def vpmc_destroy(ctx) -> None:
    load().vpmc_destroy(ctx)


def vpmc_atomic_rate(ctx, shape=(256, 256, 160), n_atomics: int = 1 << 28) -> float:
    """Non-returning int64 atomic adds per second on the context's device,
    pencil-beam track pattern over a grid of the given (nx, ny, nz)."""
    out = C.c_double(0.0)
    nx, ny, nz = shape
    _check(load().vpmc_atomic_rate(ctx, nx, ny, nz, int(n_atomics), C.byref(out)), ctx)
    return out.value


def vpmc_table_host(material: int, which: int) -> np.ndarray:
    out = np.zeros(256, np.float64)
    n = load().vpmc_table_host(material, which, _ptr(out), 256)
    if n < 0:
        _check(n)
    return out[:n]


def vpmc_load_geometry(ctx, geom: I.Geometry, hu=None, flags: int = 0) -> None:
    """hu: optional torch device tensor (with flags=DEVICE_PTRS) or numpy int16."""
    nx, ny, nz = geom.shape
    src = hu
    if src is None and geom.kind == GEOM_HU:
        src = np.ascontiguousarray(geom.hu, np.int16)
    _check(load().vpmc_load_geometry(ctx, geom.kind, _ptr(src), nx, ny, nz, _f3(geom.spacing),
                                     _f3(geom.origin), flags), ctx)


def beam_struct(b: I.Beam) -> vpmc_beam:
    s = vpmc_beam()
    s.iso_mm = _f3(b.iso)
    s.ex, s.ey, s.ez = _f3(b.ex), _f3(b.ey), _f3(b.ez)
    return s


def vpmc_set_aperture(ctx, field_id: int, field: I.Field) -> None:
    beam = beam_struct(field.beam)
    poly = None
    nv = 0
    if field.block is not None and field.polygon is not None and len(field.polygon) > 0:
        poly = np.ascontiguousarray(field.polygon, np.float32)
        nv = poly.shape[0]
    blk = None
    if field.block is not None:
        blk = vpmc_block(field.block.thickness_mm, field.block.density_gcc, field.block.downstream_mm)
    rs = None
    if field.rs is not None:
        rs = vpmc_rs(field.rs.wet_mm, field.rs.diameter_mm, field.rs.downstream_mm)
    _check(load().vpmc_set_aperture(ctx, field_id, C.byref(beam), _ptr(poly), nv,
                                    C.byref(blk) if blk is not None else None,
                                    C.byref(rs) if rs is not None else None), ctx)
    focus = field.block.focus_mm if field.block is not None else 0.0
    if field.vsad_mm or focus:
        vpmc_set_divergence(ctx, field_id, field.vsad_mm, focus)


def vpmc_set_divergence(ctx, field_id: int, vsad_mm: float, focus_mm: float) -> None:
    _check(load().vpmc_set_divergence(ctx, field_id, float(vsad_mm), float(focus_mm)), ctx)


def spot_array(spots: np.ndarray):
    arr = (vpmc_spot * max(1, len(spots)))()
    for i in range(len(spots)):
        s = arr[i]
        s.x_mm, s.y_mm = float(spots["x_mm"][i]), float(spots["y_mm"][i])
        s.energy_mev, s.sigma_mm = float(spots["energy_mev"][i]), float(spots["sigma_mm"][i])
        s.energy_sigma_mev, s.weight = float(spots["energy_sigma_mev"][i]), float(spots["weight"][i])
        s.n_histories = int(spots["n_histories"][i])
    return arr


def scenario_array(scen: Sequence[I.Scenario]):
    arr = (vpmc_scenario * len(scen))()
    for i, sc in enumerate(scen):
        arr[i].shift_mm = _f3(sc.shift_mm)
        arr[i].range_scale = float(sc.range_scale)
    return arr


def make_opts(seed=0, physics=PHYS_ALL, n_batches=0, output=OUT_DOSE, fixed_point_bits=0,
              flags=0, stream=None, max_device_bytes=0, block_threads=0, grid_blocks=0,
              hist_per_lane=0, max_slots=0, queue_cap=0) -> vpmc_opts:
    o = vpmc_opts()
    o.seed, o.physics, o.n_batches, o.output = seed, physics, n_batches, output
    o.fixed_point_bits, o.flags = fixed_point_bits, flags
    o.hip_stream = stream
    o.max_device_bytes, o.block_threads, o.grid_blocks = max_device_bytes, block_threads, grid_blocks
    o.hist_per_lane, o.max_slots, o.queue_cap = hist_per_lane, max_slots, queue_cap
    return o


def vpmc_run_spots(ctx, field_id: int, spots, n_spots: int, scen, n_scen: int, opts: vpmc_opts,
                   dose=None, sigma=None, ledger=None, row_ptr=None) -> None:
    _check(load().vpmc_run_spots(ctx, field_id, C.cast(spots, C.c_void_p) if spots is not None else None,
                                 n_spots, C.cast(scen, C.c_void_p) if scen is not None else None, n_scen,
                                 C.byref(opts), _ptr(dose), _ptr(sigma), _ptr(ledger), _ptr(row_ptr)), ctx)


def vpmc_run_spots_noalloc(ctx, field_id: int, spots, n_spots: int, scen, n_scen: int, opts: vpmc_opts,
                           dose=None, sigma=None, ledger=None) -> None:
    _check(load().vpmc_run_spots_noalloc(ctx, field_id, C.cast(spots, C.c_void_p) if spots is not None else None,
                                         n_spots, C.cast(scen, C.c_void_p) if scen is not None else None, n_scen,
                                         C.byref(opts), _ptr(dose), _ptr(sigma), _ptr(ledger)), ctx)


def vpmc_run_batched(ctx, field_ids: Sequence[int], spot_arrays: Sequence, scen, n_scen: int,
                     opts: vpmc_opts, dose=None, ledger=None, row_ptr=None) -> None:
    nf = len(field_ids)
    ids = (C.c_int * nf)(*field_ids)
    ptrs = (C.c_void_p * nf)(*[C.cast(a, C.c_void_p) for a in spot_arrays])
    ns = (C.c_int * nf)(*[len(a) for a in spot_arrays])
    _check(load().vpmc_run_batched(ctx, ids, ptrs, ns, nf, C.cast(scen, C.c_void_p), n_scen, C.byref(opts),
                                   _ptr(dose), _ptr(ledger), _ptr(row_ptr)), ctx)


def vpmc_autotune(ctx, field_id: int, spots, n_spots: int, scen, base: vpmc_opts,
                  sample_histories: int) -> vpmc_opts:
    best = vpmc_opts()
    _check(load().vpmc_autotune(ctx, field_id, C.cast(spots, C.c_void_p), n_spots, C.cast(scen, C.c_void_p),
                                C.byref(base), int(sample_histories), C.byref(best)), ctx)
    return best


def vpmc_copy_csr(ctx, col=None, val=None, q=None) -> None:
    _check(load().vpmc_copy_csr(ctx, _ptr(col), _ptr(val), _ptr(q)), ctx)


def vpmc_last_tally_k(ctx) -> int:
    """Fixed-point exponent of the last run (dense or CSR)."""
    k = C.c_int(0)
    rc = load().vpmc_last_tally(ctx, 0, None, C.byref(k), 0)
    if rc == E_STATE:   # CSR run without dense output: k is still recorded
        rc = load().vpmc_last_tally(ctx, -1, None, C.byref(k), 0)
    _check(rc, ctx)
    return k.value


def vpmc_last_let(ctx, scen_index: int, ql_out=None, flags: int = 0) -> int:
    """Copy the last dense run's LET numerator of one scenario; returns its shift."""
    sh = C.c_int(0)
    _check(load().vpmc_last_let(ctx, scen_index, _ptr(ql_out), C.byref(sh), flags), ctx)
    return sh.value


def vpmc_last_tally(ctx, scen_index: int, q_out=None, flags: int = 0) -> int:
    k = C.c_int(0)
    _check(load().vpmc_last_tally(ctx, scen_index, _ptr(q_out), C.byref(k), flags), ctx)
    return k.value


def vpmc_optimize(ctx, row_ptr, col, val, n_scen: int, n_spots: int, nvox: int, roi, x, *, d_presc: float,
                  w_target: float, d_max: float, w_oar: float, iters: int, n_power: int = 20,
                  row_stride: int = 0, row_offset: int = 0, flags: int = 0, stream=None, obj_hist=None,
                  dose=None) -> float:
    """Spot weights by projected FISTA on the scenario influence matrices; x
    (FP64, n_spots) holds the start and receives the result, obj_hist
    (iters + 1) and dose (n_scen x nvox FP32) are optional outputs.  Arrays
    are numpy (host) or torch CUDA tensors with flags |= DEVICE_PTRS.
    Returns the step constant L."""
    p = vpmc_opt_params(d_presc=float(d_presc), w_target=float(w_target), d_max=float(d_max),
                        w_oar=float(w_oar), iters=int(iters), n_power=int(n_power), row_stride=int(row_stride),
                        row_offset=int(row_offset), flags=int(flags), hip_stream=stream)
    L = C.c_double(0.0)
    _check(load().vpmc_optimize(ctx, _ptr(row_ptr), _ptr(col), _ptr(val), int(n_scen), int(n_spots), int(nvox),
                                _ptr(roi), C.byref(p), _ptr(x), _ptr(obj_hist), C.byref(L), _ptr(dose)), ctx)
    return L.value


def vpmc_csr_cells(ctx, row_ptr, col, q, k: int, cell_of_voxel, n_cells: int, flags: int = 0):
    """Rows merged into cells (dynamic voxel spacing): (row_ptr, cell, q,
    val) as numpy arrays, or torch CUDA tensors with flags |= DEVICE_PTRS."""
    n_rows = len(row_ptr) - 1
    L = load()
    if flags & DEVICE_PTRS:
        import torch
        dev = row_ptr.device
        rp_out = torch.empty(n_rows + 1, dtype=torch.int64, device=dev)
    else:
        rp_out = np.zeros(n_rows + 1, np.int64)
    _check(L.vpmc_csr_cells(ctx, _ptr(row_ptr), n_rows, _ptr(col), _ptr(q), int(k), _ptr(cell_of_voxel),
                            int(n_cells), _ptr(rp_out), None, None, None, flags), ctx)
    nout = int(rp_out[-1])
    if flags & DEVICE_PTRS:
        cell = torch.empty(nout, dtype=torch.int32, device=dev)
        qo = torch.empty(nout, dtype=torch.int64, device=dev)
        val = torch.empty(nout, dtype=torch.float32, device=dev)
    else:
        cell, qo, val = np.zeros(nout, np.int32), np.zeros(nout, np.int64), np.zeros(nout, np.float32)
    _check(L.vpmc_csr_cells(ctx, _ptr(row_ptr), n_rows, _ptr(col), _ptr(q), int(k), _ptr(cell_of_voxel),
                            int(n_cells), _ptr(rp_out), _ptr(cell), _ptr(qo), _ptr(val), flags), ctx)
    return rp_out, cell, qo, val


def vpmc_last_stats(ctx) -> dict:
    st = vpmc_stats()
    _check(load().vpmc_last_stats(ctx, C.byref(st)), ctx)
    return {f: getattr(st, f) for f, _ in vpmc_stats._fields_}


def _f32(a):
    return np.ascontiguousarray(a, np.float32)


def vpmc_surrogate_param_count() -> int:
    return load().vpmc_surrogate_param_count()


def vpmc_surrogate_set_weights(ctx, params) -> None:
    p = _f32(params)
    _check(load().vpmc_surrogate_set_weights(ctx, _ptr(p), p.size), ctx)


SURROGATE_DIMS = (8, 256, 256, 256, 256, 29)


def surrogate_init(seed: int = 0) -> np.ndarray:
    """Initial surrogate parameters: He-uniform weights (the output layer
    scaled by 0.1), zero biases; layer by layer W[out][in] then b[out]."""
    rng = np.random.default_rng(seed)
    parts = []
    for li, (ni, no) in enumerate(zip(SURROGATE_DIMS[:-1], SURROGATE_DIMS[1:])):
        lim = np.sqrt(6.0 / ni) * (0.1 if li == len(SURROGATE_DIMS) - 2 else 1.0)
        parts += [rng.uniform(-lim, lim, size=no * ni), np.zeros(no)]
    return np.concatenate(parts).astype(np.float32)


def vpmc_surrogate_config(ctx, d_fallback_mm: float = 3.0, p_lo: float = 0.02, p_hi: float = 0.98) -> None:
    _check(load().vpmc_surrogate_config(ctx, float(d_fallback_mm), float(p_lo), float(p_hi)), ctx)


def vpmc_surrogate_get_weights(ctx) -> np.ndarray:
    p = np.zeros(vpmc_surrogate_param_count(), np.float32)
    _check(load().vpmc_surrogate_get_weights(ctx, _ptr(p), p.size), ctx)
    return p


def vpmc_surrogate_load(ctx, path: Optional[str]) -> None:
    _check(load().vpmc_surrogate_load(ctx, None if path is None else os.fsencode(path)), ctx)


def vpmc_surrogate_save(ctx, path: str) -> None:
    _check(load().vpmc_surrogate_save(ctx, os.fsencode(path)), ctx)


def vpmc_surrogate_sample(ctx, field_id: int, entries, seed: int = 0, physics: int = PHYS_ALL):
    """Plain brass traversals -> (x [n,8], y [n,3], trans [n])."""
    e = _f32(entries)
    n = e.shape[0]
    x = np.zeros((n, 8), np.float32)
    y = np.zeros((n, 3), np.float32)
    t = np.zeros(n, np.float32)
    _check(load().vpmc_surrogate_sample(ctx, field_id, _ptr(e), n, seed, physics, _ptr(x), _ptr(y), _ptr(t)), ctx)
    return x, y, t


def vpmc_surrogate_forward(ctx, x) -> np.ndarray:
    x = _f32(x)
    out = np.zeros((x.shape[0], 29), np.float32)
    _check(load().vpmc_surrogate_forward(ctx, _ptr(x), x.shape[0], _ptr(out)), ctx)
    return out


def vpmc_surrogate_loss_grad(ctx, x, y, trans):
    x, y, t = _f32(x), _f32(y), _f32(trans)
    g = np.zeros(vpmc_surrogate_param_count(), np.float32)
    loss = C.c_double(0.0)
    _check(load().vpmc_surrogate_loss_grad(ctx, _ptr(x), _ptr(y), _ptr(t), x.shape[0], _ptr(g), C.byref(loss)), ctx)
    return loss.value, g


def vpmc_surrogate_train(ctx, x, y, trans, epochs: int, batch: int, lr: float, seed: int = 0) -> np.ndarray:
    x, y, t = _f32(x), _f32(y), _f32(trans)
    losses = np.zeros(epochs, np.float32)
    _check(load().vpmc_surrogate_train(ctx, _ptr(x), _ptr(y), _ptr(t), x.shape[0], epochs, batch, float(lr), seed,
                                       _ptr(losses)), ctx)
    return losses


# --------------------------------------------------------------- convenience
class Engine:
    """Owns one context on one GPU and runs Case objects through the C ABI,
    with torch tensors as device outputs on torch's current stream."""

    def __init__(self, device: int = 0):
        import torch
        self.torch = torch
        self.device = device
        # torch's runtime first: its tensors and streams are the ones passed in
        if not torch.cuda.is_available():
            raise RuntimeError("no HIP device visible to torch; the VP engine needs an MI355X GPU")
        torch.cuda.set_device(device)
        self.ctx = vpmc_create(device)
        self._geom = None

    def close(self):
        if self.ctx is not None:
            vpmc_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def load_case(self, case: I.Case) -> None:
        if self._geom is not case.geometry:
            vpmc_load_geometry(self.ctx, case.geometry)
            self._geom = case.geometry
        for fi, f in enumerate(case.fields):
            vpmc_set_aperture(self.ctx, fi, f)

    def stream_ptr(self):
        return C.c_void_p(self.torch.cuda.current_stream(self.device).cuda_stream)

    def run_dose(self, case: I.Case, field_index: int = 0, scenarios=None, n_batches: Optional[int] = None,
                 sigma: bool = True, physics: Optional[int] = None, seed: Optional[int] = None,
                 fixed_point_bits: int = 0, grid_blocks: int = 0, surrogate: bool = False, let: bool = False):
        """Dense dose of one field for the given scenario list.  Returns
        (dose[n_scen, nz, ny, nx], sigma or None, ledger_mev[n_scen, 6]) with
        dose/sigma as torch float32 tensors on the GPU.  surrogate: deep
        brass entries cross the block by the learned surrogate.  let: also
        tally the dose-averaged LET numerator (last_let)."""
        torch = self.torch
        scen = case.scenarios if scenarios is None else scenarios
        B = case.n_batches if n_batches is None else n_batches
        nx, ny, nz = case.geometry.shape
        dev = torch.device("cuda", self.device)
        dose = torch.empty((len(scen), nz, ny, nx), dtype=torch.float32, device=dev)
        sig = torch.empty_like(dose) if (sigma and B >= 2) else None
        led = np.zeros((len(scen), NLEDGER), np.float64)
        spots = case.fields[field_index].spots
        opts = make_opts(seed=case.seed if seed is None else seed,
                         physics=case.physics if physics is None else physics,
                         n_batches=B if (sigma and B >= 2) else 0, fixed_point_bits=fixed_point_bits,
                         flags=DEVICE_PTRS | (SURROGATE if surrogate else 0) | (LET if let else 0),
                         stream=self.stream_ptr(),
                         grid_blocks=grid_blocks)
        vpmc_run_spots(self.ctx, field_index, spot_array(spots), len(spots), scenario_array(scen), len(scen),
                       opts, dose, sig, led)
        return dose, sig, led

    def run_csr(self, case: I.Case, scenarios=None, fixed_point_bits: int = 0, physics: Optional[int] = None,
                seed: Optional[int] = None, hist_per_lane: int = 0, max_slots: int = 0, grid_blocks: int = 0,
                graph: bool = False, fields=None, dose: bool = False, copy: bool = True,
                device_out: bool = False, block_threads: int = 0, surrogate: bool = False, queue_cap: int = 0):
        """Influence matrices of all fields x scenarios in one batched pass.
        Rows are ordered (scenario, field, spot).  Returns (row_ptr, col, val,
        q, k) as numpy arrays (col/val/q None when copy is False), plus the
        plan dose per scenario as a torch tensor when dose is True.  With
        device_out, row_ptr, col (int32) and val (FP32 Gy) stay on the GPU as
        torch tensors and q is None.  surrogate: deep brass entries cross the
        block by the learned surrogate."""
        torch = self.torch
        self.load_case(case)
        scen = case.scenarios if scenarios is None else scenarios
        fids = list(range(len(case.fields))) if fields is None else list(fields)
        arrays = [spot_array(case.fields[f].spots) for f in fids]
        n_rows = len(scen) * sum(len(case.fields[f].spots) for f in fids)
        row_ptr = np.zeros(n_rows + 1, np.int64)
        led = np.zeros((len(scen), NLEDGER), np.float64)
        nx, ny, nz = case.geometry.shape
        d = None
        flags = (GRAPH if graph else 0) | (SURROGATE if surrogate else 0)
        if dose:
            d = torch.empty((len(scen), nz, ny, nx), dtype=torch.float32, device=torch.device("cuda", self.device))
        opts = make_opts(seed=case.seed if seed is None else seed,
                         physics=case.physics if physics is None else physics, output=OUT_CSR,
                         fixed_point_bits=fixed_point_bits, flags=flags, stream=self.stream_ptr(),
                         hist_per_lane=hist_per_lane, max_slots=max_slots, grid_blocks=grid_blocks,
                         block_threads=block_threads, queue_cap=queue_cap)
        if device_out:
            opts.flags |= DEVICE_PTRS
            dev = torch.device("cuda", self.device)
            rp_dev = torch.empty(n_rows + 1, dtype=torch.int64, device=dev)
            vpmc_run_batched(self.ctx, fids, arrays, scenario_array(scen), len(scen), opts, d, led, rp_dev)
            nnz = int(rp_dev[-1].item())
            colt = torch.empty(nnz, dtype=torch.int32, device=dev)
            valt = torch.empty(nnz, dtype=torch.float32, device=dev)
            vpmc_copy_csr(self.ctx, colt, valt, None)
            self.last_ledger = led
            k = vpmc_last_tally_k(self.ctx)
            if dose:
                return rp_dev, colt, valt, None, k, d
            return rp_dev, colt, valt, None, k
        if dose:
            # device dose needs device pointers for every output
            opts.flags |= DEVICE_PTRS
            rp_dev = torch.empty(n_rows + 1, dtype=torch.int64, device=torch.device("cuda", self.device))
            vpmc_run_batched(self.ctx, fids, arrays, scenario_array(scen), len(scen), opts, d, led, rp_dev)
            row_ptr = rp_dev.cpu().numpy()
        else:
            vpmc_run_batched(self.ctx, fids, arrays, scenario_array(scen), len(scen), opts, None, led, row_ptr)
        k = vpmc_last_tally_k(self.ctx)
        col = val = q = None
        if copy:
            nnz = int(row_ptr[-1])
            if opts.flags & DEVICE_PTRS:
                dev = torch.device("cuda", self.device)
                colt = torch.empty(nnz, dtype=torch.int32, device=dev)
                valt = torch.empty(nnz, dtype=torch.float32, device=dev)
                qt = torch.empty(nnz, dtype=torch.int64, device=dev)
                vpmc_copy_csr(self.ctx, colt, valt, qt)
                col, val, q = colt.cpu().numpy(), valt.cpu().numpy(), qt.cpu().numpy()
            else:
                col = np.zeros(nnz, np.int32)
                val = np.zeros(nnz, np.float32)
                q = np.zeros(nnz, np.int64)
                vpmc_copy_csr(self.ctx, col, val, q)
        self.last_ledger = led
        if dose:
            return row_ptr, col, val, q, k, d
        return row_ptr, col, val, q, k

    def train_surrogate(self, case: I.Case, field_index: int = 0, n: int = 2_000_000, epochs: int = 6,
                        batch: int = 4096, lr: float = 1e-3, seed: int = 0, fields=None):
        """Train the aperture surrogate on the GPU: n entry states near the
        polygon edges of the given fields (default: field_index only;
        energies 71-229 MeV) cross their block with the plain transport,
        then Adam over the brass entries.  Returns the mean loss per epoch."""
        self.load_case(case)
        fids = [field_index] if fields is None else list(fields)
        xs, ys, ts = [], [], []
        for j, fi in enumerate(fids):
            m = n // len(fids) + (1 if j < n % len(fids) else 0)
            xy, ang, e = I.surrogate_training_entries(m, seed=seed + 7919 * j, polygon=case.fields[fi].polygon)
            ent = np.column_stack([xy, ang, e]).astype(np.float32)
            x, y, t = vpmc_surrogate_sample(self.ctx, fi, ent, seed=seed + 1 + j)
            keep = t >= 0
            xs.append(x[keep]); ys.append(y[keep]); ts.append(t[keep])
        vpmc_surrogate_set_weights(self.ctx, surrogate_init(seed))
        return vpmc_surrogate_train(self.ctx, np.concatenate(xs), np.concatenate(ys), np.concatenate(ts), epochs,
                                    batch, lr, seed)

    def optimize(self, rp, col, val, n_scen: int, spots_per_field, nvox: int, roi, *, d_presc: float,
                 w_target: float = 1.0, d_max: float, w_oar: float = 1.0, iters: int = 80, n_power: int = 20,
                 mode: str = "MFO", x0=None, reuse: bool = False):
        """Robust spot weights from the influence matrices of vpmc_run_batched
        (rows ordered scenario, field, spot; torch CUDA tensors).  MFO: all
        fields' spots together against d_presc.  SFO: every field alone
        against d_presc / n_fields (its rows addressed inside the whole
        layout).  Returns (x [spots], step constants)."""
        torch = self.torch
        dev = torch.device("cuda", self.device)
        counts = [int(n) for n in spots_per_field]
        total = sum(counts)
        x = (torch.ones(total, dtype=torch.float64, device=dev) if x0 is None
             else torch.as_tensor(x0, dtype=torch.float64, device=dev).clone())
        flags = DEVICE_PTRS | (OPT_REUSE if reuse else 0)
        common = dict(w_target=w_target, d_max=d_max, w_oar=w_oar, iters=iters, n_power=n_power,
                      flags=flags, stream=self.stream_ptr())
        if mode == "MFO":
            L = vpmc_optimize(self.ctx, rp, col, val, n_scen, total, nvox, roi, x, d_presc=d_presc, **common)
            return x, [L]
        if mode != "SFO":
            raise ValueError("mode is MFO or SFO")
        Ls, off = [], 0
        common["flags"] = DEVICE_PTRS          # each field builds its own index
        for n in counts:
            xf = x[off:off + n].contiguous()
            Ls.append(vpmc_optimize(self.ctx, rp, col, val, n_scen, n, nvox, roi, xf,
                                    d_presc=d_presc / len(counts), row_stride=total, row_offset=off, **common))
            x[off:off + n] = xf
            off += n
        return x, Ls

    def last_let(self, scen_index: int = 0):
        """(numerator int64[nz, ny, nx] on the GPU, shift) of the last dense
        run with let=True; LET_d = numerator * 2^shift / last_tally q."""
        torch = self.torch
        ql = torch.empty(self._geom.nvox, dtype=torch.int64, device=torch.device("cuda", self.device))
        sh = vpmc_last_let(self.ctx, scen_index, ql, DEVICE_PTRS)
        nx, ny, nz = self._geom.shape
        return ql.reshape(nz, ny, nx), sh

    def last_tally(self, scen_index: int = 0):
        torch = self.torch
        nvox = self._geom.nvox
        q = torch.empty(nvox, dtype=torch.int64, device=torch.device("cuda", self.device))
        k = vpmc_last_tally(self.ctx, scen_index, q, DEVICE_PTRS)
        nx, ny, nz = self._geom.shape
        return q.reshape(nz, ny, nx), k
