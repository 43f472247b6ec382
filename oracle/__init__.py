"""ctypes wrapper of the FP64 history-based oracle.

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the
CPU-baseline leg of the benchmark.  The HIP library never calls it.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

from . import build as _build

HERE = os.path.dirname(os.path.abspath(__file__))
MAX_ELEM = 8

GAMMA, ELECTRON, POSITRON = 0, 1, 2
LIM_PHYS, LIM_ELOSS, LIM_GEOM, LIM_FIELD = 0, 1, 2, 3
PROC_NAMES = ["compton", "pair", "moller", "bhabha", "brems_em", "brems_ep", "annihilation", "null"]
NPROC = len(PROC_NAMES)
COUNTER_NAMES = (["steps_gamma", "steps_electron", "steps_positron",
                  "tracks_gamma", "tracks_electron", "tracks_positron"]
                 + ["proc_" + p for p in PROC_NAMES]
                 + ["escaped", "killed", "rejection_exhausted", "trace_dropped",
                    "rk_substeps", "rk_rejected"])
LEDGER_NAMES = ["escaped", "killed", "n_pair", "n_annih"]
# single steps ended after one stage (Sec. 2.1.2): ComputeIntLen, GeomQuery,
# Propagation, multiple scattering, continuous loss; 0 = the whole step
STOP_LIMIT, STOP_GEOM, STOP_MOVE, STOP_MSC, STOP_ELOSS = 1, 2, 3, 4, 5
TABLE_NAMES = ["compton", "pair", "moller", "brems_em", "S_em", "R_em",
               "bhabha", "brems_ep", "S_ep", "R_ep"]
PDG_TO_TYPE = {22: GAMMA, 11: ELECTRON, -11: POSITRON}


class Material(C.Structure):
    _fields_ = [("density", C.c_double), ("n_elem", C.c_int32), ("Z", C.c_int32 * MAX_ELEM),
                ("A", C.c_double * MAX_ELEM), ("w", C.c_double * MAX_ELEM),
                ("I_elem_eV", C.c_double * MAX_ELEM), ("I_eV", C.c_double), ("X0_cm", C.c_double)]


class Geometry(C.Structure):
    _fields_ = [("axis", C.c_int32), ("n_vol", C.c_int32), ("bounds", C.POINTER(C.c_double)),
                ("material", C.POINTER(C.c_int32)), ("cell", C.POINTER(C.c_int32)),
                ("env", C.c_double * 2), ("world", C.c_double * 4), ("B", C.c_double * 3),
                ("field_map", C.c_int32), ("pad", C.c_int32), ("sol", C.c_double * 2)]


class Field(C.Structure):
    _fields_ = [("map", C.c_int32), ("pad", C.c_int32), ("B", C.c_double * 3), ("sol", C.c_double * 2)]


class Config(C.Structure):
    _fields_ = [("e_min", C.c_double), ("bins_per_decade", C.c_double), ("n_nodes", C.c_int32),
                ("field_method", C.c_int32), ("t_cut", C.c_double), ("k_cut", C.c_double),
                ("t_track", C.c_double), ("chord_tol", C.c_double), ("push", C.c_double),
                ("rk_frac", C.c_double), ("max_steps", C.c_int64), ("fs_alias", C.c_int32), ("pad", C.c_int32),
                ("rk_tol", C.c_double), ("rk_max_sub", C.c_int32), ("pad2", C.c_int32)]

MAP_UNIFORM, MAP_SOLENOID = 0, 1
FIELD_HELIX, FIELD_RK4, FIELD_RK45 = 0, 1, 2


TRACE_DTYPE = np.dtype([("tid", "<u8"), ("event", "<u4"), ("nstep", "<u4"), ("type", "<i4"),
                        ("limiter", "<i4"), ("vol_pre", "<i4"), ("vol_post", "<i4"),
                        ("process", "<i4"), ("n_children", "<i4"), ("pos", "<f8", (3,)),
                        ("dir", "<f8", (3,)), ("ekin", "<f8"), ("edep", "<f8"), ("step", "<f8")])
assert TRACE_DTYPE.itemsize == 112

_lib = None


def load(rebuild: bool = False):
    global _lib
    if _lib is not None and not rebuild:
        return _lib
    if rebuild or not os.path.exists(_build.LIB):
        _build.build()
    lib = C.CDLL(_build.LIB)
    dp, ip, up32, up64, lp = (C.POINTER(C.c_double), C.POINTER(C.c_int32), C.POINTER(C.c_uint32),
                              C.POINTER(C.c_uint64), C.POINTER(C.c_int64))
    lib.or_setup.argtypes = [C.POINTER(Material), C.c_int32, C.POINTER(Geometry), C.POINTER(Config)]
    lib.or_error.restype = C.c_char_p
    lib.or_transport.argtypes = [C.c_void_p, C.c_int64, C.c_uint64, C.c_int32, dp, dp, lp,
                                 C.c_void_p, C.c_int64, lp]
    lib.or_single_step.argtypes = [C.c_int64, C.c_uint64, ip, dp, dp, dp, up32, up64, up32,
                                   dp, dp, dp, dp, ip, ip, ip, ip, ip, ip, ip, dp, dp, up64,
                                   dp, dp, dp, dp]
    lib.or_stage_step.argtypes = [C.c_int32, C.c_int64, C.c_uint64, ip, dp, dp, dp, up32, up64, up32,
                                  dp, dp, dp, dp, ip, ip, ip, ip, ip, ip, ip, dp, dp, up64,
                                  dp, dp, dp, dp, dp]
    lib.or_philox4x32_10.argtypes = [up32, up32, up32]
    lib.or_stream.argtypes = [C.c_uint64, C.c_uint32, C.c_uint64, C.c_uint32, C.c_uint32, up32]
    for name in ["or_u53", "or_expo"]:
        getattr(lib, name).argtypes = [C.c_uint32, C.c_uint32]
        getattr(lib, name).restype = C.c_double
    lib.or_u32.argtypes = [C.c_uint32]
    lib.or_u32.restype = C.c_double
    for name in ["or_mat_electron_density", "or_mat_X0", "or_mat_I", "or_mat_plasma_energy"]:
        getattr(lib, name).argtypes = [C.c_int32]
        getattr(lib, name).restype = C.c_double
    lib.or_xs_compton_per_electron.argtypes = [C.c_double]
    lib.or_xs_compton_per_electron.restype = C.c_double
    for name in ["or_xs_compton", "or_xs_pair", "or_xs_brems", "or_xs_moller", "or_xs_bhabha",
                 "or_density_effect"]:
        getattr(lib, name).argtypes = [C.c_int32, C.c_double]
        getattr(lib, name).restype = C.c_double
    lib.or_dedx_col.argtypes = [C.c_int32, C.c_double, C.c_int32, C.c_double]
    lib.or_dedx_col.restype = C.c_double
    lib.or_dedx_rad.argtypes = [C.c_int32, C.c_double, C.c_double]
    lib.or_dedx_rad.restype = C.c_double
    lib.or_dedx_total.argtypes = [C.c_int32, C.c_double, C.c_int32]
    lib.or_dedx_total.restype = C.c_double
    lib.or_n_nodes.restype = C.c_int32
    lib.or_node_energy.argtypes = [C.c_int32]
    lib.or_node_energy.restype = C.c_double
    lib.or_table_node.argtypes = [C.c_int32, C.c_int32, C.c_int32]
    lib.or_table_node.restype = C.c_double
    lib.or_table_value.argtypes = [C.c_int32, C.c_int32, C.c_double]
    lib.or_table_value.restype = C.c_double
    lib.or_range_inverse.argtypes = [C.c_int32, C.c_int32, C.c_double]
    lib.or_range_inverse.restype = C.c_double
    lib.or_locate.argtypes = [dp]
    lib.or_locate.restype = C.c_int32
    lib.or_dist_out.argtypes = [C.c_int32, dp, dp, ip]
    lib.or_dist_out.restype = C.c_double
    lib.or_safety.argtypes = [C.c_int32, dp]
    lib.or_safety.restype = C.c_double
    lib.or_helix_move.argtypes = [C.c_int32, C.c_double, dp, C.c_double, dp, dp]
    lib.or_rk4_move.argtypes = [C.c_int32, C.c_double, dp, C.c_double, C.c_int32, dp, dp]
    fp = C.POINTER(Field)
    lib.or_field_eval.argtypes = [fp, dp, dp]
    lib.or_rk4_field_move.argtypes = [C.c_int32, C.c_double, fp, C.c_double, C.c_int32, dp, dp]
    lib.or_rk45_move.argtypes = [C.c_int32, C.c_double, fp, C.c_double, C.c_double, C.c_int32,
                                 dp, dp, dp, ip]
    lib.or_rk45_move.restype = C.c_int32
    lib.or_dp45_tableau.argtypes = [dp, dp, dp, dp]
    lib.or_highland.argtypes = [C.c_int32, C.c_double, C.c_double]
    lib.or_highland.restype = C.c_double
    lib.or_rotate.argtypes = [dp, C.c_double, C.c_double, C.c_double]
    for name in ["or_sample_compton", "or_sample_pair", "or_sample_brems", "or_sample_moller",
                 "or_sample_bhabha"]:
        for nm in (name, name + "_alias"):
            getattr(lib, nm).argtypes = [C.c_double, C.c_uint64, C.c_uint32, C.c_uint64, C.c_uint32, dp]
            getattr(lib, nm).restype = C.c_int
    lib.or_escape_hist.argtypes = [C.c_void_p]
    lib.or_alias_node_energy.argtypes = [C.c_int32]
    lib.or_alias_node_energy.restype = C.c_double
    lib.or_alias_table.argtypes = [C.c_int32, C.c_int32, dp, dp, ip]
    lib.or_alias_table.restype = C.c_int32
    lib.or_alias_pdf.argtypes = [C.c_int32, C.c_double, C.c_double]
    lib.or_alias_pdf.restype = C.c_double
    lib.or_alias_var.argtypes = [C.c_int32, C.c_double, C.c_double]
    lib.or_alias_var.restype = C.c_double
    lib.or_alias_xi.argtypes = [C.c_int32, C.c_double, dp]
    lib.or_alias_xi.restype = C.c_double
    _lib = lib
    return lib


def _ptr(a, ct):
    return a.ctypes.data_as(C.POINTER(ct))


def make_material(md) -> Material:
    m = Material()
    m.density = md["density"]
    els = md["elements"]
    m.n_elem = len(els)
    for j, (Z, A, w, I) in enumerate(els):
        m.Z[j] = Z
        m.A[j] = A
        m.w[j] = w
        m.I_elem_eV[j] = I
    m.I_eV = md.get("I_eV", 0.0)
    m.X0_cm = md.get("X0_cm", 0.0)
    return m


class Oracle:
    """One configured oracle context (the library holds a single global one)."""

    def __init__(self, geom, table_spec=None, run_spec=None):
        import gv_inputs
        self.lib = load()
        ts = dict(gv_inputs.TABLE_SPEC)
        ts.update(table_spec or {})
        rs = dict(gv_inputs.RUN_SPEC)
        rs.update(run_spec or {})
        self.geom = geom
        mats = geom["materials"]
        arr = (Material * len(mats))(*[make_material(md) for md in mats])
        self._bounds = np.ascontiguousarray(geom["bounds"], dtype=np.float64)
        self._mat = np.ascontiguousarray(geom["material"], dtype=np.int32)
        self._cell = np.ascontiguousarray(geom["cell"], dtype=np.int32)
        g = Geometry()
        g.axis = geom["axis"]
        g.n_vol = len(self._mat)
        g.bounds = _ptr(self._bounds, C.c_double)
        g.material = _ptr(self._mat, C.c_int32)
        g.cell = _ptr(self._cell, C.c_int32)
        for i in range(2):
            g.env[i] = float(geom["env"][i])
        for i in range(4):
            g.world[i] = float(geom["world"][i])
        for i in range(3):
            g.B[i] = float(geom["B"][i])
        g.field_map = int(geom.get("field_map", MAP_UNIFORM))
        sol = geom.get("sol", (0.0, 0.0))
        g.sol[0], g.sol[1] = float(sol[0]), float(sol[1])
        cfg = Config()
        cfg.e_min = ts["e_min"]
        cfg.bins_per_decade = ts["bins_per_decade"]
        cfg.n_nodes = ts["n_nodes"]
        cfg.t_cut = ts["t_cut"]
        cfg.k_cut = ts["k_cut"]
        cfg.t_track = ts["t_track"]
        cfg.chord_tol = rs["chord_tol"]
        cfg.push = rs["push"]
        cfg.rk_frac = rs["rk_frac"]
        cfg.max_steps = rs["max_steps"]
        cfg.field_method = rs["field_method"]
        cfg.fs_alias = rs.get("fs_alias", 0)
        cfg.rk_tol = rs["rk_tol"]
        cfg.rk_max_sub = rs["rk_max_sub"]
        rc = self.lib.or_setup(arr, len(mats), C.byref(g), C.byref(cfg))
        if rc != 0:
            raise RuntimeError("oracle setup failed: " + self.lib.or_error().decode())
        self.n_cells = int(max(self._cell.max() + 1, 0))
        self.n_mats = len(mats)

    # ---- full transport ----
    def transport(self, primaries, seed, n_threads=None, trace_cap=0):
        prim = np.ascontiguousarray(primaries)
        n = len(prim)
        n_events = int(prim["event"].max()) + 1
        edep = np.zeros((n_events, self.n_cells), dtype=np.float64)
        ledger = np.zeros((n_events, 4), dtype=np.float64)
        counters = np.zeros(len(COUNTER_NAMES), dtype=np.int64)
        if n_threads is None:
            n_threads = min(os.cpu_count() or 1, 16)
        tn = np.zeros(1, dtype=np.int64)
        trace = np.zeros(trace_cap, dtype=TRACE_DTYPE) if trace_cap else None
        rc = self.lib.or_transport(prim.ctypes.data, n, seed, n_threads, _ptr(edep, C.c_double),
                                   _ptr(ledger, C.c_double), _ptr(counters, C.c_int64),
                                   trace.ctypes.data if trace is not None else None, trace_cap,
                                   _ptr(tn, C.c_int64))
        if rc != 0:
            raise RuntimeError("oracle transport failed: " + self.lib.or_error().decode())
        hist = np.zeros((3, 40, 20), dtype=np.int64)
        self.lib.or_escape_hist(hist.ctypes.data)
        out = dict(edep=edep, ledger=ledger, counters=dict(zip(COUNTER_NAMES, counters.tolist())),
                   escape_hist=hist)
        if trace is not None:
            out["trace"] = trace[: int(tn[0])]
        return out

    # ---- one step of independent tracks ----
    def single_step(self, st, seed, stop=0):
        """One step of each state; stop = STOP_LIMIT ... STOP_ELOSS ends it
        after that stage of Sec. 2.1.2 (the per-stage reference)."""
        n = len(st["type"])
        f64 = lambda *s: np.zeros(s, dtype=np.float64)
        i32 = lambda *s: np.zeros(s, dtype=np.int32)
        o = dict(pos=f64(n, 3), dir=f64(n, 3), ekin=f64(n), edep=f64(n), vol=i32(n), vol_pre=i32(n),
                 limiter=i32(n), process=i32(n), status=i32(n), n_children=i32(n),
                 ch_type=i32(n, 2), ch_ekin=f64(n, 2), ch_dir=f64(n, 2, 3),
                 ch_tid=np.zeros((n, 2), dtype=np.uint64), step=f64(n), s_phys=f64(n),
                 d_bnd=f64(n), safety=f64(n), s_eloss=f64(n))
        typ = np.ascontiguousarray(st["type"], dtype=np.int32)
        pos = np.ascontiguousarray(st["pos"], dtype=np.float64)
        dr = np.ascontiguousarray(st["dir"], dtype=np.float64)
        ek = np.ascontiguousarray(st["ekin"], dtype=np.float64)
        ev = np.ascontiguousarray(st["event"], dtype=np.uint32)
        tid = np.ascontiguousarray(st["tid"], dtype=np.uint64)
        ns = np.ascontiguousarray(st["nstep"], dtype=np.uint32)
        d, i, u32, u64 = C.c_double, C.c_int32, C.c_uint32, C.c_uint64
        rc = self.lib.or_stage_step(
            stop, n, seed, _ptr(typ, i), _ptr(pos, d), _ptr(dr, d), _ptr(ek, d), _ptr(ev, u32),
            _ptr(tid, u64), _ptr(ns, u32), _ptr(o["pos"], d), _ptr(o["dir"], d), _ptr(o["ekin"], d),
            _ptr(o["edep"], d), _ptr(o["vol"], i), _ptr(o["vol_pre"], i), _ptr(o["limiter"], i),
            _ptr(o["process"], i), _ptr(o["status"], i), _ptr(o["n_children"], i),
            _ptr(o["ch_type"], i), _ptr(o["ch_ekin"], d), _ptr(o["ch_dir"], d), _ptr(o["ch_tid"], u64),
            _ptr(o["step"], d), _ptr(o["s_phys"], d), _ptr(o["d_bnd"], d), _ptr(o["safety"], d),
            _ptr(o["s_eloss"], d))
        if rc != 0:
            raise RuntimeError("oracle single step failed: " + self.lib.or_error().decode())
        return o

    # ---- unit access ----
    def table(self, m, which):
        w = TABLE_NAMES.index(which) if isinstance(which, str) else which
        n = self.lib.or_n_nodes()
        return np.array([self.lib.or_table_node(m, w, i) for i in range(n)])

    def nodes(self):
        n = self.lib.or_n_nodes()
        return np.array([self.lib.or_node_energy(i) for i in range(n)])

    def table_value(self, m, which, T):
        w = TABLE_NAMES.index(which) if isinstance(which, str) else which
        return self.lib.or_table_value(m, w, T)

    def locate(self, p):
        p = np.ascontiguousarray(p, dtype=np.float64)
        return self.lib.or_locate(_ptr(p, C.c_double))

    def dist_out(self, vol, p, d):
        p = np.ascontiguousarray(p, dtype=np.float64)
        d = np.ascontiguousarray(d, dtype=np.float64)
        nx = C.c_int32(0)
        t = self.lib.or_dist_out(vol, _ptr(p, C.c_double), _ptr(d, C.c_double), C.byref(nx))
        return t, nx.value

    def safety(self, vol, p):
        p = np.ascontiguousarray(p, dtype=np.float64)
        return self.lib.or_safety(vol, _ptr(p, C.c_double))


def philox(ctr, key):
    lib = load()
    c = (C.c_uint32 * 4)(*ctr)
    k = (C.c_uint32 * 2)(*key)
    o = (C.c_uint32 * 4)()
    lib.or_philox4x32_10(c, k, o)
    return list(o)


def stream(seed, event, tid, nstep, purpose):
    lib = load()
    o = (C.c_uint32 * 4)()
    lib.or_stream(seed, event, tid, nstep, purpose, o)
    return list(o)


def make_field(map_kind=MAP_UNIFORM, B=(0.0, 0.0, 0.0), sol=(0.0, 0.0)) -> Field:
    f = Field()
    f.map = map_kind
    for i in range(3):
        f.B[i] = float(B[i])
    f.sol[0], f.sol[1] = float(sol[0]), float(sol[1])
    return f


def field_eval(field: Field, x):
    lib = load()
    xa = np.ascontiguousarray(x, dtype=np.float64)
    out = np.zeros(3)
    lib.or_field_eval(C.byref(field), _ptr(xa, C.c_double), _ptr(out, C.c_double))
    return out


def rk45_move(type_, ekin, field: Field, s, tol, max_sub, pos, direction):
    """Adaptive Dormand-Prince move; returns (pos, dir, s_done, n_accepted, n_rejected)."""
    lib = load()
    p = np.array(pos, dtype=np.float64)
    d = np.array(direction, dtype=np.float64)
    sd = C.c_double()
    nr = C.c_int32()
    na = lib.or_rk45_move(type_, ekin, C.byref(field), s, tol, max_sub, _ptr(p, C.c_double),
                          _ptr(d, C.c_double), C.byref(sd), C.byref(nr))
    return p, d, sd.value, int(na), int(nr.value)


def rk4_field_move(type_, ekin, field: Field, s, nsub, pos, direction):
    lib = load()
    p = np.array(pos, dtype=np.float64)
    d = np.array(direction, dtype=np.float64)
    lib.or_rk4_field_move(type_, ekin, C.byref(field), s, nsub, _ptr(p, C.c_double), _ptr(d, C.c_double))
    return p, d


def helix_move(type_, ekin, B, s, pos, direction):
    lib = load()
    Ba = np.ascontiguousarray(B, dtype=np.float64)
    p = np.array(pos, dtype=np.float64)
    d = np.array(direction, dtype=np.float64)
    lib.or_helix_move(type_, ekin, _ptr(Ba, C.c_double), s, _ptr(p, C.c_double), _ptr(d, C.c_double))
    return p, d


def dp45_tableau():
    lib = load()
    a = np.zeros(49)
    b = np.zeros(7)
    bh = np.zeros(7)
    c = np.zeros(7)
    lib.or_dp45_tableau(_ptr(a, C.c_double), _ptr(b, C.c_double), _ptr(bh, C.c_double), _ptr(c, C.c_double))
    return a.reshape(7, 7), b, bh, c
