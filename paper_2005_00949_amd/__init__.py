"""Thin ctypes binding of libgv.so, the gfx950 basketised EM-shower stepping
library (C ABI in include/gv.h).  Argument marshalling only: every step of the
transport runs in the library's HIP kernels.  Importing this module never
falls back to anything else: if the library is missing, `load()` raises.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "_build", "libgv.so")

GV_OK = 0
STATUS_NAMES = {0: "GV_OK", 1: "GV_E_INVALID_ARG", 2: "GV_E_GEOMETRY", 3: "GV_E_TABLES", 4: "GV_E_HIP",
                5: "GV_E_NOT_INIT", 6: "GV_E_CAPACITY", 7: "GV_E_STATE"}
DRIVER_PLAIN, DRIVER_BATCHED = 0, 1
P64, PMIX = 0, 1
FIELD_HELIX, FIELD_RK4, FIELD_RK45 = 0, 1, 2
MAP_UNIFORM, MAP_SOLENOID = 0, 1
ORDER_ARRIVAL, ORDER_STABLE = 0, 1
DEPOSIT_FLOAT, DEPOSIT_FIXED = 0, 1
FS_COMPTON, FS_PAIR, FS_BREMS, FS_MOLLER, FS_BHABHA = 0, 1, 2, 3, 4
FS_ALL = 31
DBG_STEP, DBG_PHILOX, DBG_COMPACT, DBG_TABLE, DBG_GEOM = 0, 1, 2, 3, 4
# the step ended after one of its stages (Sec. 2.1.2)
DBG_THRU_LIMIT, DBG_THRU_GEOM, DBG_THRU_MOVE, DBG_THRU_MSC, DBG_THRU_ELOSS = 5, 6, 7, 8, 9
MAX_ELEM = 8
PROC_NAMES = ["compton", "pair", "moller", "bhabha", "brems_em", "brems_ep", "annihilation", "null"]
# table ids for DBG_TABLE: type * 4 + column, 12 = node energies
TABLE_IDS = {"compton": 0, "pair": 1, "moller": 4, "brems_em": 5, "S_em": 6, "R_em": 7,
             "bhabha": 8, "brems_ep": 9, "S_ep": 10, "R_ep": 11, "nodes": 12}


class GvError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{STATUS_NAMES.get(code, code)}: {msg}")
        self.code = code


class Material(C.Structure):
    _fields_ = [("density", C.c_double), ("n_elem", C.c_int32), ("Z", C.c_int32 * MAX_ELEM),
                ("A", C.c_double * MAX_ELEM), ("w", C.c_double * MAX_ELEM),
                ("I_elem_eV", C.c_double * MAX_ELEM), ("I_eV", C.c_double), ("X0_cm", C.c_double)]


class Geometry(C.Structure):
    _fields_ = [("axis", C.c_int32), ("n_vol", C.c_int32), ("bounds", C.POINTER(C.c_double)),
                ("material", C.POINTER(C.c_int32)), ("cell", C.POINTER(C.c_int32)),
                ("env", C.c_double * 2), ("world", C.c_double * 4), ("B", C.c_double * 3),
                ("field_map", C.c_int32), ("reserved", C.c_int32), ("sol_cm", C.c_double * 2)]


class Tables(C.Structure):
    _fields_ = [("e_min_MeV", C.c_double), ("bins_per_decade", C.c_double), ("n_nodes", C.c_int32),
                ("reserved", C.c_int32), ("t_cut_MeV", C.c_double), ("k_cut_MeV", C.c_double),
                ("t_track_MeV", C.c_double)]


class Config(C.Structure):
    _fields_ = [("driver", C.c_int32), ("precision", C.c_int32), ("basket", C.c_int32),
                ("occupancy", C.c_int32), ("inner_steps", C.c_int32), ("graph_steps", C.c_int32),
                ("field_method", C.c_int32), ("edep_on_device", C.c_int32),
                ("max_steps_per_track", C.c_int64), ("capacity", C.c_int64),
                ("max_events_in_flight", C.c_int64), ("chord_tol_cm", C.c_double),
                ("push_cm", C.c_double), ("rk_frac", C.c_double), ("hip_stream", C.c_void_p),
                ("trace_cap", C.c_int64), ("queue_order", C.c_int32), ("deposit_mode", C.c_int32),
                ("fs_alias", C.c_int32), ("reserved2", C.c_int32),
                ("rk_tol", C.c_double), ("rk_max_substeps", C.c_int32), ("reserved3", C.c_int32)]


class Stats(C.Structure):
    _fields_ = [("steps", C.c_int64 * 3), ("tracks", C.c_int64 * 3), ("interactions", C.c_int64 * 8),
                ("escaped", C.c_int64), ("killed", C.c_int64), ("rejection_exhausted", C.c_int64),
                ("iterations", C.c_int64), ("graph_replays", C.c_int64), ("trace_records", C.c_int64),
                ("overflow_restarts", C.c_int64),
                ("e_in", C.c_double), ("e_dep", C.c_double), ("e_escaped", C.c_double),
                ("e_killed", C.c_double), ("n_pair", C.c_double), ("n_annih", C.c_double),
                ("transport_ms", C.c_double), ("init_ms", C.c_double), ("kernel_ms", C.c_double),
                ("kernel_launches", C.c_int64), ("alg_bytes", C.c_double),
                ("driver", C.c_int32), ("precision", C.c_int32), ("basket", C.c_int32),
                ("occupancy", C.c_int32), ("inner_steps", C.c_int32), ("graph_steps", C.c_int32),
                ("capacity", C.c_int64), ("state_bytes", C.c_double), ("autotune_ms", C.c_double),
                ("tuned", C.c_int32), ("queue_order", C.c_int32), ("reserved", C.c_int32),
                ("tail_kernel_ms", C.c_double),
                ("rk_substeps", C.c_int64), ("rk_rejected", C.c_int64), ("rk_lane_slots", C.c_int64),
                ("lane_slots", C.c_int64), ("tail_steps", C.c_int64),
                ("helper_steps", C.c_int64), ("rk_parked", C.c_int64)]


class DebugIO(C.Structure):
    _fields_ = [("precision", C.c_int32), ("block", C.c_int32), ("material", C.c_int32),
                ("which", C.c_int32), ("seed", C.c_uint64)] + [
        (name, C.c_void_p) for name in
        ["type", "pos_in", "dir_in", "ekin_in", "event", "tid", "nstep", "vol_in", "words", "codes",
         "pos", "dir", "ekin", "edep", "vol", "vol_pre", "limiter", "process", "status", "n_children",
         "ch_type", "ch_ekin", "ch_dir", "ch_tid", "step", "s_phys", "d_bnd", "safety", "words_out",
         "index", "counts", "values", "s_eloss"]]


TRACE_DTYPE = np.dtype([("tid", "<u8"), ("event", "<u4"), ("nstep", "<u4"), ("type", "<i4"),
                        ("limiter", "<i4"), ("vol_pre", "<i4"), ("vol_post", "<i4"),
                        ("process", "<i4"), ("n_children", "<i4"), ("pos", "<f8", (3,)),
                        ("dir", "<f8", (3,)), ("ekin", "<f8"), ("edep", "<f8"), ("step", "<f8")])
assert TRACE_DTYPE.itemsize == 112

_lib = None


def load():
    """Load libgv.so; raise if it has not been built (no fallback exists)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with paper_2005_00949_amd/build.py "
                          "(there is no fallback path)")
    lib = C.CDLL(LIB_PATH)
    lib.gv_last_error.restype = C.c_char_p
    lib.gv_init.argtypes = [C.POINTER(Material), C.c_int32, C.POINTER(Geometry), C.POINTER(Tables)]
    lib.gv_configure.argtypes = [C.POINTER(Config)]
    lib.gv_transport.argtypes = [C.c_void_p, C.c_int64, C.c_uint64, C.c_void_p]
    lib.gv_stage.argtypes = [C.c_void_p, C.c_int64]
    lib.gv_transport_staged.argtypes = [C.c_uint64, C.c_void_p]
    lib.gv_stats.argtypes = [C.POINTER(Stats)]
    lib.gv_ledger.argtypes = [C.c_void_p, C.c_int64]
    lib.gv_trace.argtypes = [C.c_void_p, C.c_int64, C.POINTER(C.c_int64)]
    lib.gv_n_cells.argtypes = [C.POINTER(C.c_int32)]
    lib.gv_finalize.restype = None
    lib.gv_debug_step.argtypes = [C.c_int32, C.c_int64, C.POINTER(DebugIO)]
    lib.gv_alias_table.argtypes = [C.c_int32, C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]
    lib.gv_escape_hist.argtypes = [C.c_void_p, C.c_int64]
    lib.gv_compact3_noalloc.argtypes = [C.c_void_p, C.c_int64, C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p]
    _lib = lib
    return lib


def _check(rc):
    if rc != GV_OK:
        raise GvError(rc, _lib.gv_last_error().decode())


def _material(md) -> Material:
    m = Material()
    m.density = md["density"]
    els = md["elements"]
    m.n_elem = len(els)
    for j, (Z, A, w, I) in enumerate(els):
        m.Z[j], m.A[j], m.w[j], m.I_elem_eV[j] = Z, A, w, I
    m.I_eV = md.get("I_eV", 0.0)
    m.X0_cm = md.get("X0_cm", 0.0)
    return m


def _p(a):
    return a.ctypes.data if a is not None else None


def compact3_noalloc(codes_ptr, n, block, index_ptr, counts_ptr, stream=None):
    """gv_compact3_noalloc on device buffers given as raw device pointers
    (codes: 3n int8, index: 9n int32, counts: 4 uint32); enqueued on
    `stream` (a hipStream_t as an integer, or None for the null stream)."""
    lib = load()
    _check(lib.gv_compact3_noalloc(C.c_void_p(codes_ptr), n, block, C.c_void_p(index_ptr), C.c_void_p(counts_ptr),
                                   C.c_void_p(stream) if stream else None))


class Engine:
    """The library's single context: gv_init + gv_configure + gv_transport."""

    def __init__(self, geom, table_spec=None, **config):
        import gv_inputs
        self.lib = load()
        ts = dict(gv_inputs.TABLE_SPEC)
        ts.update(table_spec or {})
        mats = geom["materials"]
        arr = (Material * len(mats))(*[_material(md) for md in mats])
        self._bounds = np.ascontiguousarray(geom["bounds"], dtype=np.float64)
        self._mat = np.ascontiguousarray(geom["material"], dtype=np.int32)
        self._cell = np.ascontiguousarray(geom["cell"], dtype=np.int32)
        g = Geometry()
        g.axis = geom["axis"]
        g.n_vol = len(self._mat)
        g.bounds = self._bounds.ctypes.data_as(C.POINTER(C.c_double))
        g.material = self._mat.ctypes.data_as(C.POINTER(C.c_int32))
        g.cell = self._cell.ctypes.data_as(C.POINTER(C.c_int32))
        for i in range(2):
            g.env[i] = float(geom["env"][i])
        for i in range(4):
            g.world[i] = float(geom["world"][i])
        for i in range(3):
            g.B[i] = float(geom["B"][i])
        g.field_map = int(geom.get("field_map", MAP_UNIFORM))
        sol = geom.get("sol", (0.0, 0.0))
        g.sol_cm[0], g.sol_cm[1] = float(sol[0]), float(sol[1])
        t = Tables(ts["e_min"], ts["bins_per_decade"], ts["n_nodes"], 0, ts["t_cut"], ts["k_cut"],
                   ts["t_track"])
        _check(self.lib.gv_init(arr, len(mats), C.byref(g), C.byref(t)))
        nc = C.c_int32()
        _check(self.lib.gv_n_cells(C.byref(nc)))
        self.n_cells = nc.value
        self.geom = geom
        self.config = dict(driver=DRIVER_BATCHED, precision=PMIX, basket=0, occupancy=0, inner_steps=0,
                           graph_steps=0, field_method=FIELD_HELIX, edep_on_device=0,
                           max_steps_per_track=1 << 20, capacity=0, max_events_in_flight=0,
                           chord_tol_cm=1e-3, push_cm=1e-7, rk_frac=0.05, hip_stream=None, trace_cap=0,
                           queue_order=ORDER_ARRIVAL, deposit_mode=DEPOSIT_FLOAT, fs_alias=0,
                           rk_tol=0.0, rk_max_substeps=0)
        self.configure(**config)

    def configure(self, **kw):
        unknown = set(kw) - set(self.config)
        if unknown:
            raise TypeError(f"unknown options {sorted(unknown)}")
        old = dict(self.config)
        self.config.update(kw)
        c = Config(**{k: v for k, v in self.config.items()})
        try:
            _check(self.lib.gv_configure(C.byref(c)))
        except GvError:
            self.config = old          # the library keeps its previous configuration too
            raise

    def transport(self, primaries, seed, edep_out=None):
        """primaries: gv_inputs.PRIMARY_DTYPE array.  Returns edep [events, cells]
        (numpy, host) unless edep_out (a device pointer, edep_on_device=1) is given."""
        prim = np.ascontiguousarray(primaries)
        n_events = int(prim["event"].max()) + 1
        if edep_out is None:
            edep = np.zeros((n_events, self.n_cells), dtype=np.float64)
            _check(self.lib.gv_transport(prim.ctypes.data, len(prim), seed, edep.ctypes.data))
            self.n_events = n_events
            return edep
        _check(self.lib.gv_transport(prim.ctypes.data, len(prim), seed, edep_out))
        self.n_events = n_events
        return None

    def stage(self, primaries):
        """Validate and copy the primaries to the device once (gv_stage)."""
        prim = np.ascontiguousarray(primaries)
        _check(self.lib.gv_stage(prim.ctypes.data, len(prim)))
        self.n_events = int(prim["event"].max()) + 1
        self._staged = prim

    def transport_staged(self, seed, edep_out=None):
        """Transport the staged batch (gv_transport_staged); edep_out as in transport()."""
        if edep_out is None:
            edep = np.zeros((self.n_events, self.n_cells), dtype=np.float64)
            _check(self.lib.gv_transport_staged(seed, edep.ctypes.data))
            return edep
        _check(self.lib.gv_transport_staged(seed, edep_out))
        return None

    def stats(self):
        s = Stats()
        _check(self.lib.gv_stats(C.byref(s)))
        out = {}
        for name, _ in Stats._fields_:
            v = getattr(s, name)
            out[name] = list(v) if hasattr(v, "__len__") else v
        out["total_steps"] = sum(out["steps"])
        return out

    def ledger(self):
        L = np.zeros((self.n_events, 4), dtype=np.float64)
        _check(self.lib.gv_ledger(L.ctypes.data, self.n_events))
        return L

    def trace(self):
        cap = self.config["trace_cap"]
        tr = np.zeros(cap, dtype=TRACE_DTYPE)
        n = C.c_int64()
        _check(self.lib.gv_trace(tr.ctypes.data, cap, C.byref(n)))
        return tr[: n.value]

    # ---- test entry points ----
    def _debug(self, stage, n, io):
        _check(self.lib.gv_debug_step(stage, n, C.byref(io)))

    def debug_step(self, st, seed, precision=P64, stage=DBG_STEP):
        """One step of each state (stage = DBG_STEP), or the step ended after
        one of its stages (stage = DBG_THRU_LIMIT ... DBG_THRU_ELOSS, which
        also return s_eloss)."""
        n = len(st["type"])
        f64 = lambda *s: np.zeros(s, dtype=np.float64)
        i32 = lambda *s: np.zeros(s, dtype=np.int32)
        o = dict(pos=f64(n, 3), dir=f64(n, 3), ekin=f64(n), edep=f64(n), vol=i32(n), vol_pre=i32(n),
                 limiter=i32(n), process=i32(n), status=i32(n), n_children=i32(n), ch_type=i32(n, 2),
                 ch_ekin=f64(n, 2), ch_dir=f64(n, 2, 3), ch_tid=np.zeros((n, 2), np.uint64),
                 step=f64(n), s_phys=f64(n), d_bnd=f64(n), safety=f64(n))
        if stage != DBG_STEP:
            o["s_eloss"] = f64(n)
        keep = dict(type=np.ascontiguousarray(st["type"], np.int32),
                    pos_in=np.ascontiguousarray(st["pos"], np.float64),
                    dir_in=np.ascontiguousarray(st["dir"], np.float64),
                    ekin_in=np.ascontiguousarray(st["ekin"], np.float64),
                    event=np.ascontiguousarray(st["event"], np.uint32),
                    tid=np.ascontiguousarray(st["tid"], np.uint64),
                    nstep=np.ascontiguousarray(st["nstep"], np.uint32))
        io = DebugIO()
        io.precision = precision
        io.seed = seed
        for k, v in keep.items():
            setattr(io, k, _p(v))
        io.pos, io.dir, io.ekin, io.edep = _p(o["pos"]), _p(o["dir"]), _p(o["ekin"]), _p(o["edep"])
        io.vol, io.vol_pre, io.limiter, io.process = _p(o["vol"]), _p(o["vol_pre"]), _p(o["limiter"]), _p(o["process"])
        io.status, io.n_children, io.ch_type = _p(o["status"]), _p(o["n_children"]), _p(o["ch_type"])
        io.ch_ekin, io.ch_dir, io.ch_tid = _p(o["ch_ekin"]), _p(o["ch_dir"]), _p(o["ch_tid"])
        io.step, io.s_phys, io.d_bnd, io.safety = _p(o["step"]), _p(o["s_phys"]), _p(o["d_bnd"]), _p(o["safety"])
        if stage != DBG_STEP:
            io.s_eloss = _p(o["s_eloss"])
        self._debug(stage, n, io)
        return o

    def debug_philox(self, words):
        w = np.ascontiguousarray(words, dtype=np.uint32).reshape(-1, 6)
        out = np.zeros((len(w), 4), dtype=np.uint32)
        io = DebugIO()
        io.words, io.words_out = _p(w), _p(out)
        self._debug(DBG_PHILOX, len(w), io)
        return out

    def debug_compact(self, codes, block=256):
        c = np.ascontiguousarray(codes, dtype=np.int8).reshape(-1, 3)
        n = len(c)
        index = np.zeros(9 * n, dtype=np.int32)
        counts = np.zeros(3, dtype=np.int64)
        io = DebugIO()
        io.codes, io.index, io.counts, io.block = _p(c), _p(index), _p(counts), block
        self._debug(DBG_COMPACT, n, io)
        idx = index.reshape(3, 3 * n)
        return [idx[q, : counts[q]] for q in range(3)]

    def debug_table(self, material, which, precision=P64):
        w = TABLE_IDS[which] if isinstance(which, str) else which
        n = 801 if which != "nodes" else 801
        vals = np.zeros(4096, dtype=np.float64)
        io = DebugIO()
        io.material, io.which, io.precision, io.values = material, w, precision, _p(vals)
        from gv_inputs import TABLE_SPEC
        n = TABLE_SPEC["n_nodes"]
        self._debug(DBG_TABLE, n, io)
        return vals[:n].copy()

    def debug_geom(self, pos, dirs, vol=None):
        p = np.ascontiguousarray(pos, dtype=np.float64).reshape(-1, 3)
        d = np.ascontiguousarray(dirs, dtype=np.float64).reshape(-1, 3)
        n = len(p)
        v = np.full(n, -2, np.int32) if vol is None else np.ascontiguousarray(vol, dtype=np.int32)
        out = dict(d_bnd=np.zeros(n), next=np.zeros(n, np.int32), vol=np.zeros(n, np.int32),
                   safety=np.zeros(n))
        io = DebugIO()
        io.pos_in, io.dir_in, io.vol_in = _p(p), _p(d), _p(v)
        io.d_bnd, io.vol, io.vol_pre, io.safety = _p(out["d_bnd"]), _p(out["next"]), _p(out["vol"]), _p(out["safety"])
        self._debug(DBG_GEOM, n, io)
        return out

    def escape_hist(self):
        """Escaping particles of the last transport: counts [type, energy bin, cos bin]."""
        h = np.zeros((3, 40, 20), dtype=np.uint64)
        _check(self.lib.gv_escape_hist(h.ctypes.data, h.size))
        return h.astype(np.int64)

    def alias_table(self, model, node):
        """Final-state table of one model at one node: (valid, p, q, alias)."""
        p, q = np.zeros(65), np.zeros(64)
        a, v = np.zeros(64, dtype=np.int32), np.zeros(1, dtype=np.int32)
        _check(self.lib.gv_alias_table(model, node, p.ctypes.data, q.ctypes.data, a.ctypes.data, v.ctypes.data))
        return bool(v[0]), p, q, a

    def close(self):
        self.lib.gv_finalize()
