"""Thin Python binding of libpic (ctypes). Argument marshalling only: every step of the
deposition, sorting and gather runs in the HIP library; torch provides device memory and
the current stream. Names follow include/pic.h.
"""
import ctypes
import os

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpic.so")

PIC_OK = 0
(PIC_ERR_INVALID_ARG, PIC_ERR_UNSUPPORTED, PIC_ERR_OUT_OF_DOMAIN, PIC_ERR_CAPACITY,
 PIC_ERR_INVALID_PARTICLE, PIC_ERR_HIP) = -1, -2, -3, -4, -5, -6
PIC_BC_PERIODIC, PIC_BC_GUARD = 0, 1
PATH_AUTO, PATH_ATOMIC, PATH_CELL_VALU, PATH_MFMA_BF16, PATH_MFMA_FP16, PATH_UNSORTED = range(6)
PATH_NAMES = {"auto": PATH_AUTO, "atomic": PATH_ATOMIC, "cell_valu": PATH_CELL_VALU,
              "mfma_bf16": PATH_MFMA_BF16, "mfma_fp16": PATH_MFMA_FP16, "unsorted": PATH_UNSORTED}
REBIN_FULL, REBIN_INCREMENTAL, REBIN_AUTO = 0, 1, 2
F_ACCUMULATE, F_EMIT_MOVERS, F_DRIFT, F_MIDPOINT = 1, 4, 8, 16
INVALID_ID = -1

EXPORTS = ["pic_sort_policy_default", "pic_policy_decide", "pic_bins_create", "pic_bins_destroy",
           "pic_bins_get_view", "pic_bins_copy_tables", "pic_rebin", "pic_rebin_stats_read",
           "pic_rebin_history", "pic_bins_report_perf",
           "pic_deposit", "pic_deposit_noalloc", "pic_deposit_rho", "pic_gather_fields", "pic_deposit_backward",
           "pic_drift", "pic_push", "pic_deposit_esirkepov",
           "pic_plan_create",
           "pic_plan_destroy", "pic_deposit_batched", "pic_plan_info", "pic_plan_patch_path",
           "pic_tuning_load", "pic_auto_path", "pic_check", "pic_last_error"]


class PicError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"libpic status {status}: {msg}")
        self.status = status


class PicGrid(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int), ("n", ctypes.c_int * 3), ("x0", ctypes.c_double * 3),
                ("dx", ctypes.c_double * 3), ("inv_dx", ctypes.c_double * 3),
                ("bc", ctypes.c_int * 3), ("ng", ctypes.c_int), ("order", ctypes.c_int),
                ("q", ctypes.c_float), ("dt", ctypes.c_double)]


class PicParticles(ctypes.Structure):
    _fields_ = [("nslots", ctypes.c_int64)] + [(k, ctypes.c_void_p) for k in
                                              ("x", "y", "z", "ux", "uy", "uz", "w", "id")]


class PicSortPolicy(ctypes.Structure):
    _fields_ = [("min_interval", ctypes.c_int), ("interval", ctypes.c_int),
                ("rebuild_count", ctypes.c_int), ("empty_ratio", ctypes.c_double),
                ("full_ratio", ctypes.c_double), ("perf_enable", ctypes.c_int),
                ("perf_degrad", ctypes.c_double)]


class PicRebinStats(ctypes.Structure):
    _fields_ = [("n_valid", ctypes.c_int64), ("n_moved", ctypes.c_int64),
                ("n_overflow", ctypes.c_int64), ("n_mover_drop", ctypes.c_int64),
                ("n_local_rebuilds", ctypes.c_int32), ("n_global_sorts", ctypes.c_int32),
                ("empty_slot_ratio", ctypes.c_double), ("global_sort_recommended", ctypes.c_int32),
                ("last_mode", ctypes.c_int32), ("error_flags", ctypes.c_uint32)]


class PicRebinRecord(ctypes.Structure):
    _fields_ = [("seq", ctypes.c_int64), ("mode", ctypes.c_int32), ("trigger", ctypes.c_int32),
                ("steps_since_sort", ctypes.c_int32), ("rebuilds_since_sort", ctypes.c_int32),
                ("known_empty_ratio", ctypes.c_double), ("n_valid", ctypes.c_int64),
                ("n_moved", ctypes.c_int64), ("n_overflow", ctypes.c_int64),
                ("n_mover_drop", ctypes.c_int64), ("n_local_rebuilds", ctypes.c_int32),
                ("error_flags", ctypes.c_uint32), ("empty_slot_ratio", ctypes.c_double),
                ("complete", ctypes.c_int32), ("pad", ctypes.c_int32)]


POLICY_LAG = 2


class PicBinsView(ctypes.Structure):
    _fields_ = [("nbins", ctypes.c_int64), ("ntiles", ctypes.c_int64), ("ntile", ctypes.c_int32 * 3),
                ("off", ctypes.c_void_p), ("len", ctypes.c_void_p), ("bin_cell", ctypes.c_void_p)]


_lib = None


def lib():
    """Load libpic.so; fails loudly if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_2601_08277_amd/build_lib.py")
    L = ctypes.CDLL(LIB_PATH)
    vp, i32, i64, dbl, u32 = ctypes.c_void_p, ctypes.c_int, ctypes.c_int64, ctypes.c_double, ctypes.c_uint
    P = ctypes.POINTER
    L.pic_last_error.restype = ctypes.c_char_p
    L.pic_sort_policy_default.argtypes = [P(PicSortPolicy)]
    L.pic_sort_policy_default.restype = None
    L.pic_policy_decide.argtypes = [P(PicSortPolicy), i32, i32, dbl, dbl, dbl, P(ctypes.c_int)]
    L.pic_policy_decide.restype = i32
    L.pic_bins_create.argtypes = [P(PicGrid), P(ctypes.c_int), dbl, i64, i64, P(vp)]
    L.pic_bins_destroy.argtypes = [vp]
    L.pic_bins_get_view.argtypes = [vp, P(PicBinsView)]
    L.pic_bins_copy_tables.argtypes = [vp, vp, vp, vp, vp]
    L.pic_rebin.argtypes = [P(PicGrid), P(PicParticles), vp, i32, P(PicSortPolicy), vp]
    L.pic_rebin_stats_read.argtypes = [vp, vp, P(PicRebinStats)]
    L.pic_rebin_history.argtypes = [vp, vp, i64, ctypes.c_int32, P(PicRebinRecord),
                                    P(ctypes.c_int32)]
    L.pic_bins_report_perf.argtypes = [vp, dbl]
    L.pic_deposit.argtypes = [P(PicGrid), P(PicParticles), vp, vp, vp, vp, i32, u32, vp]
    L.pic_deposit_noalloc.argtypes = [P(PicGrid), P(PicParticles), vp, vp, vp, vp, i32, u32, vp]
    L.pic_deposit_backward.argtypes = [P(PicGrid), P(PicParticles), vp, vp, vp, vp, vp, vp, vp,
                                       vp, vp, vp, vp, u32, vp]
    L.pic_drift.argtypes = [P(PicGrid), P(PicParticles), dbl, vp]
    L.pic_push.argtypes = [P(PicGrid), P(PicParticles), vp] + [vp] * 6 + [dbl, dbl, u32, vp]
    L.pic_deposit_esirkepov.argtypes = [P(PicGrid), P(PicParticles), vp] + [vp] * 6 + [u32, vp]
    L.pic_plan_create.argtypes = [P(PicGrid), i32, P(vp), ctypes.c_char_p, P(vp)]
    L.pic_plan_destroy.argtypes = [vp]
    L.pic_deposit_batched.argtypes = [vp, P(PicParticles), P(vp), i32, u32, vp]
    L.pic_check.argtypes = [vp, vp]
    L.pic_tuning_load.argtypes = [ctypes.c_char_p]
    L.pic_auto_path.argtypes = [P(PicGrid), vp]
    L.pic_plan_patch_path.argtypes = [vp, i32, P(ctypes.c_int)]
    for name in EXPORTS:
        if name not in ("pic_last_error", "pic_sort_policy_default", "pic_policy_decide"):
            getattr(L, name).restype = i32
    _lib = L
    return L


def _check(status):
    if status != PIC_OK:
        raise PicError(status, lib().pic_last_error().decode())


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


class Grid:
    """Grid descriptor built from a params dict (see synth.py)."""

    def __init__(self, params):
        self.params = dict(params)
        p = self.params
        g = PicGrid()
        g.dim = p["dim"]
        n = tuple(p["n"]) + (1,) * (3 - len(p["n"]))
        for d in range(3):
            g.n[d] = int(n[d]) if d < p["dim"] else 1
            g.x0[d] = p.get("x0", (0.0,) * 3)[d]
            g.dx[d] = p.get("dx", (1.0,) * 3)[d]
            g.inv_dx[d] = 1.0 / g.dx[d]
            g.bc[d] = p.get("bc", (0,) * 3)[d]
        g.ng = p.get("ng", 0)
        g.order = p["order"]
        g.q = p["q"]
        g.dt = p.get("dt", 0.0)
        self.c = g

    @property
    def dim(self):
        return self.c.dim

    @property
    def shape(self):
        """Shape of one J component, slowest dimension first."""
        N = []
        for d in range(self.c.dim):
            N.append(self.c.n[d] + (2 * self.c.ng if self.c.bc[d] == PIC_BC_GUARD else 0))
        return tuple(reversed(N))


class Particles:
    """SoA particle arrays on the GPU with `nslots` slots (valid particles first)."""

    FIELDS = (("x", torch.float64), ("y", torch.float64), ("z", torch.float64),
              ("ux", torch.float32), ("uy", torch.float32), ("uz", torch.float32),
              ("w", torch.float32), ("id", torch.int32))

    def __init__(self, nslots, device="cuda"):
        self.nslots = int(nslots)
        self.generation = 0    # bumped by every binding call that moves or rewrites slots
        for name, dt in self.FIELDS:
            fill = INVALID_ID if name == "id" else 0
            setattr(self, name, torch.full((self.nslots,), fill, dtype=dt, device=device))

    @classmethod
    def from_arrays(cls, arrays, nslots=None, device="cuda"):
        n = arrays["x"].shape[0]
        obj = cls(nslots if nslots is not None else n, device)
        if n > obj.nslots:
            raise ValueError("more particles than slots")
        for name, _ in cls.FIELDS:
            getattr(obj, name)[:n].copy_(torch.from_numpy(np.ascontiguousarray(arrays[name])))
        return obj

    def to_numpy(self):
        return {name: getattr(self, name).cpu().numpy() for name, _ in self.FIELDS}

    def c(self):
        s = PicParticles()
        s.nslots = self.nslots
        for name, _ in self.FIELDS:
            setattr(s, name, getattr(self, name).data_ptr())
        return s


def slots_for(n_particles, n_cells, slack):
    """Slots a full sort needs: particles + ceil(slack * count) per cell, with margin."""
    return int(n_particles + np.ceil(slack * n_particles) + n_cells + 1024)


class Bins:
    def __init__(self, grid, tile, slack, nslots, max_movers=0):
        self.grid = grid
        h = ctypes.c_void_p()
        t = (ctypes.c_int * 3)(*tile)
        _check(lib().pic_bins_create(ctypes.byref(grid.c), t, slack, nslots, max_movers,
                                     ctypes.byref(h)))
        self.h = h

    def close(self):
        if self.h:
            lib().pic_bins_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def view(self):
        v = PicBinsView()
        _check(lib().pic_bins_get_view(self.h, ctypes.byref(v)))
        return v

    def tables(self):
        """(off, len, bin_cell) as host numpy arrays (synchronises)."""
        v = self.view()
        nb = v.nbins
        off = np.empty(nb + 1, np.int32)
        ln = np.empty(nb, np.int32)
        bc = np.empty(nb, np.int32)
        _check(lib().pic_bins_copy_tables(self.h, off.ctypes.data, ln.ctypes.data,
                                          bc.ctypes.data, _stream()))
        return off, ln, bc

    def stats(self):
        s = PicRebinStats()
        _check(lib().pic_rebin_stats_read(self.h, _stream(), ctypes.byref(s)))
        return {k: getattr(s, k) for k, _ in PicRebinStats._fields_}

    def history(self, first=0, max_records=1 << 16):
        """Per-call rebin records (pic_rebin_history) as a list of dicts (synchronises)."""
        buf = (PicRebinRecord * max_records)()
        n = ctypes.c_int32(0)
        _check(lib().pic_rebin_history(self.h, _stream(), int(first), int(max_records), buf,
                                       ctypes.byref(n)))
        return [{k: getattr(buf[i], k) for k, _ in PicRebinRecord._fields_ if k != "pad"}
                for i in range(n.value)]

    def check(self):
        _check(lib().pic_check(self.h, _stream()))

    def report_perf(self, perf):
        _check(lib().pic_bins_report_perf(self.h, float(perf)))


def tuning_load(path):
    """Load the autotuner's cache as PIC_PATH_AUTO's density rule (None clears it)."""
    _check(lib().pic_tuning_load(path.encode() if path else None))


def auto_path(grid, bins):
    """The path PIC_PATH_AUTO would take for these bins, as a name."""
    p = lib().pic_auto_path(ctypes.byref(grid.c), bins.h)
    return {v: k for k, v in PATH_NAMES.items()}[p]


def check_nobins():
    _check(lib().pic_check(None, _stream()))


def policy(**kw):
    p = PicSortPolicy()
    lib().pic_sort_policy_default(ctypes.byref(p))
    for k, v in kw.items():
        setattr(p, k, v)
    return p


def policy_decide(steps, rebuilds, empty_ratio, perf=0.0, base=0.0, pol=None):
    trig = ctypes.c_int(0)
    d = lib().pic_policy_decide(ctypes.byref(pol) if pol is not None else None, steps, rebuilds,
                                empty_ratio, perf, base, ctypes.byref(trig))
    return bool(d), trig.value


def rebin(grid, parts, bins, mode=REBIN_INCREMENTAL, pol=None):
    parts.generation += 1
    pc = parts.c()
    _check(lib().pic_rebin(ctypes.byref(grid.c), ctypes.byref(pc), bins.h, mode,
                           ctypes.byref(pol) if pol is not None else None, _stream()))


def new_J(grid, device="cuda"):
    return [torch.empty(grid.shape, dtype=torch.float32, device=device) for _ in range(3)]


def deposit(grid, parts, bins, path=PATH_AUTO, flags=0, J=None):
    if isinstance(path, str):
        path = PATH_NAMES[path]
    if J is None:
        J = new_J(grid)
    if flags & F_DRIFT:
        parts.generation += 1
    pc = parts.c()
    _check(lib().pic_deposit(ctypes.byref(grid.c), ctypes.byref(pc), bins.h if bins else None,
                             _ptr(J[0]), _ptr(J[1]), _ptr(J[2]), path, flags, _stream()))
    return J


def deposit_noalloc(grid, parts, bins, path=PATH_AUTO, flags=0, J=None):
    """pic_deposit_noalloc: as deposit(), with the tile windows in the library's fixed
    device array (no allocation by the library)."""
    if isinstance(path, str):
        path = PATH_NAMES[path]
    if J is None:
        J = new_J(grid)
    if flags & F_DRIFT:
        parts.generation += 1
    pc = parts.c()
    _check(lib().pic_deposit_noalloc(ctypes.byref(grid.c), ctypes.byref(pc),
                                     bins.h if bins else None, _ptr(J[0]), _ptr(J[1]),
                                     _ptr(J[2]), path, flags, _stream()))
    return J


class Plan:
    """Batched deposition plan over independent 3D patches (pic_plan_create)."""

    def __init__(self, grids, bins, tune_cache=None):
        self.grids = list(grids)
        self.bins = list(bins)
        n = len(self.grids)
        garr = (PicGrid * n)(*[g.c for g in self.grids])
        barr = (ctypes.c_void_p * n)(*[b.h.value for b in self.bins])
        h = ctypes.c_void_p()
        path = tune_cache.encode() if tune_cache else None
        _check(lib().pic_plan_create(garr, n, barr, path, ctypes.byref(h)))
        self.h = h

    def info(self):
        ni, nb, bpc = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
        lds = ctypes.c_int64()
        _check(lib().pic_plan_info(self.h, ctypes.byref(ni), ctypes.byref(nb), ctypes.byref(bpc),
                                   ctypes.byref(lds)))
        return {"items": ni.value, "blocks": nb.value, "blocks_per_cu": bpc.value,
                "lds_bytes": lds.value}

    def patch_path(self, k):
        v = ctypes.c_int()
        _check(lib().pic_plan_patch_path(self.h, int(k), ctypes.byref(v)))
        return {v_: k_ for k_, v_ in PATH_NAMES.items()}[v.value]

    def close(self):
        if self.h:
            lib().pic_plan_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def deposit_batched(plan, parts_list, J_list=None, path=PATH_AUTO, flags=0):
    """Deposit every patch of `plan` in one persistent launch; returns the J lists."""
    if isinstance(path, str):
        path = PATH_NAMES[path]
    n = len(parts_list)
    if J_list is None:
        J_list = [new_J(g) for g in plan.grids]
    if flags & F_DRIFT:
        for p in parts_list:
            p.generation += 1
    parr = (PicParticles * n)(*[p.c() for p in parts_list])
    jarr = (ctypes.c_void_p * (3 * n))(*[J[c].data_ptr() for J in J_list for c in range(3)])
    _check(lib().pic_deposit_batched(plan.h, parr, jarr, path, flags, _stream()))
    return J_list


def deposit_rho(grid, parts, bins, flags=0, rho=None):
    """Charge density on the grid (pic_deposit_rho); returns the rho tensor."""
    if rho is None:
        rho = torch.empty(grid.shape, dtype=torch.float32, device=parts.x.device)
    pc = parts.c()
    _check(lib().pic_deposit_rho(ctypes.byref(grid.c), ctypes.byref(pc), bins.h, _ptr(rho),
                                 flags, _stream()))
    return rho


def gather_fields(grid, parts, bins, E, B):
    """E and B at every slot (pic_gather_fields): two lists of three float32 tensors."""
    n = parts.nslots
    dev = parts.x.device
    out = [torch.empty(n, dtype=torch.float32, device=dev) for _ in range(6)]
    F = [f.contiguous() for f in list(E) + list(B)]
    pc = parts.c()
    _check(lib().pic_gather_fields(ctypes.byref(grid.c), ctypes.byref(pc),
                                   bins.h if bins else None, *[_ptr(f) for f in F],
                                   *[_ptr(o) for o in out], _stream()))
    return out[:3], out[3:]


def push(grid, parts, bins, E, B, qm, dt):
    """Boris push in place (pic_push): gather E, B, rotate u, move x by dt."""
    F = [f.contiguous() for f in list(E) + list(B)]
    parts.generation += 1
    pc = parts.c()
    _check(lib().pic_push(ctypes.byref(grid.c), ctypes.byref(pc), bins.h if bins else None,
                          *[_ptr(f) for f in F], float(qm), float(dt), 0, _stream()))


def deposit_esirkepov(grid, parts, bins, old, flags=0, J=None):
    """Charge-conserving current (pic_deposit_esirkepov) of the move from `old` (three
    float64 tensors in slot order) to the particles' current positions in grid.dt."""
    if J is None:
        J = new_J(grid)
    oc = [o.contiguous() for o in old]
    pc = parts.c()
    _check(lib().pic_deposit_esirkepov(ctypes.byref(grid.c), ctypes.byref(pc),
                                       bins.h if bins else None, *[_ptr(o) for o in oc],
                                       _ptr(J[0]), _ptr(J[1]), _ptr(J[2]), flags, _stream()))
    return J


def deposit_backward(grid, parts, bins, G, want_dw=True):
    n = parts.nslots
    dev = parts.x.device
    out = {k: torch.empty(n, dtype=torch.float32, device=dev)
           for k in ("dx", "dy", "dz", "dux", "duy", "duz")}
    out["dw"] = torch.empty(n, dtype=torch.float32, device=dev) if want_dw else None
    Gc = [g.contiguous() for g in G]
    pc = parts.c()
    _check(lib().pic_deposit_backward(ctypes.byref(grid.c), ctypes.byref(pc),
                                      bins.h if bins else None, _ptr(Gc[0]), _ptr(Gc[1]),
                                      _ptr(Gc[2]), _ptr(out["dx"]), _ptr(out["dy"]),
                                      _ptr(out["dz"]), _ptr(out["dux"]), _ptr(out["duy"]),
                                      _ptr(out["duz"]), _ptr(out["dw"]), 0, _stream()))
    return out


def drift(grid, parts, dt):
    parts.generation += 1
    pc = parts.c()
    _check(lib().pic_drift(ctypes.byref(grid.c), ctypes.byref(pc), float(dt), _stream()))


class PicDeposit(torch.autograd.Function):
    """J = deposit(x, y, z, ux, uy, uz, w); backward through pic_deposit_backward.

    The forward saves only its inputs; shape weights are recomputed in the backward kernel.
    The particle tensors are those of a Particles object (`parts`), whose id array marks gaps.
    The backward reads the particles as they are when it runs, so it refuses to run after
    any call that moved or rewrote them (rebin, drift, push, a drifting deposit) or after an
    in-place change of the tensors: it would return gradients for other positions or another
    slot order.
    """

    @staticmethod
    def _stamp(parts):
        return (parts.generation,) + tuple(getattr(parts, n)._version for n, _ in Particles.FIELDS)

    @staticmethod
    def forward(ctx, x, y, z, ux, uy, uz, w, grid, parts, bins, path):
        ctx.grid, ctx.parts, ctx.bins = grid, parts, bins
        J = deposit(grid, parts, bins, path)
        ctx.stamp = PicDeposit._stamp(parts)
        return tuple(J)

    @staticmethod
    def backward(ctx, gJx, gJy, gJz):
        if PicDeposit._stamp(ctx.parts) != ctx.stamp:
            raise RuntimeError("PicDeposit.backward: the particles were moved or changed "
                               "after the forward; run the forward again")
        g = deposit_backward(ctx.grid, ctx.parts, ctx.bins, [gJx, gJy, gJz])
        dz = g["dz"].double() if ctx.grid.dim == 3 else torch.zeros_like(ctx.parts.z)
        return (g["dx"].double(), g["dy"].double(), dz, g["dux"], g["duy"], g["duz"], g["dw"],
                None, None, None, None)


def deposit_autograd(grid, parts, bins, path=PATH_AUTO):
    return PicDeposit.apply(parts.x, parts.y, parts.z, parts.ux, parts.uy, parts.uz, parts.w,
                            grid, parts, bins, path)
