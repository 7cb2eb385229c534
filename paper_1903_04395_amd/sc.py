"""ctypes binding for libsc (include/sc.h): argument marshalling only.

Every step of the counting runs in libsc's HIP kernels; this module converts
numpy arrays and Python values to the C ABI's plain pointers and back.  It
raises ``RuntimeError`` when the built library is missing -- there is no CPU
fallback.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

__all__ = [
    "SC_OK", "SC_EINVAL", "SC_ENOMEM", "SC_EDEVICE", "SC_ENOTFOUND", "SC_EBUSY", "SC_ESTATE",
    "SC_OPT_MAX_BATCH", "SC_OPT_GRAPH", "SC_OPT_SEGMENT", "SC_OPT_REORDER", "SC_OPT_INTERLEAVE",
    "SC_OPT_LDS_MAX", "SC_OPT_WAVE_ROW_MAX", "SC_OPT_CHAIN", "OPTION_DEFAULTS", "ScError", "PlanInfo", "KernelStat", "Launch",
    "Job", "Tune", "ServeCfg", "Query", "Result", "ServeStats", "lib", "lib_path", "sc_version",
    "sc_plan_template",
    "sc_colorset_rank", "sc_color_of", "Context",
    "Estimate", "SC_EST_BOUND", "SC_EST_SAMPLE", "SC_ABL_FASCIA", "SC_ABL_PFASCIA", "colorings_for",
    "SC_MAX_T", "SC_STATIC_SCRATCH_BYTES",
]

SC_OK, SC_EINVAL, SC_ENOMEM, SC_EDEVICE, SC_ENOTFOUND, SC_EBUSY, SC_ESTATE = 0, -1, -2, -3, -4, -5, -6
SC_OPT_MAX_BATCH, SC_OPT_GRAPH, SC_OPT_SEGMENT, SC_OPT_REORDER = 1, 3, 5, 8
SC_OPT_INTERLEAVE, SC_OPT_LDS_MAX, SC_OPT_WAVE_ROW_MAX, SC_OPT_CHAIN = 9, 10, 11, 12
SC_MAX_T = 16
SC_STATIC_SCRATCH_BYTES = 64 << 20     # the allocation-free entry point's device array

_HERE = os.path.dirname(os.path.abspath(__file__))
lib_path = os.path.join(_HERE, "libsc.so")
_lib = None

_i64p = ctypes.POINTER(ctypes.c_int64)
_i32p = ctypes.POINTER(ctypes.c_int32)
_u64p = ctypes.POINTER(ctypes.c_uint64)
_u8p = ctypes.POINTER(ctypes.c_uint8)
_dblp = ctypes.POINTER(ctypes.c_double)
_vp = ctypes.c_void_p

ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p, ctypes.c_void_p)
FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p, ctypes.c_void_p)


class PlanInfo(ctypes.Structure):
    _fields_ = [
        ("t", ctypes.c_int32), ("k", ctypes.c_int32), ("root", ctypes.c_int32),
        ("n_steps", ctypes.c_int32),
        ("child_ptr", ctypes.c_int32 * (SC_MAX_T + 1)),
        ("child_idx", ctypes.c_int32 * SC_MAX_T),
        ("step_h", ctypes.c_int32 * SC_MAX_T),
        ("step_a", ctypes.c_int32 * SC_MAX_T),
        ("step_p", ctypes.c_int32 * SC_MAX_T),
        ("step_mode", ctypes.c_int32 * SC_MAX_T),
        ("batch", ctypes.c_int32),
        ("interleave", ctypes.c_int32),
        ("arena_bytes", ctypes.c_uint64),
        ("spmm_updates", ctypes.c_double),
        ("ema_updates", ctypes.c_double),
        ("lemma1_ops", ctypes.c_double),
        ("exec_updates", ctypes.c_double),
        ("compulsory_bytes", ctypes.c_double),
        ("automorphisms", ctypes.c_double),
    ]

    def children(self):
        """Ordered children lists of the rooted template (the plan)."""
        return [list(self.child_idx[self.child_ptr[u]:self.child_ptr[u + 1]]) for u in range(self.t)]

    def steps(self):
        return [(self.step_h[i], self.step_a[i], self.step_p[i]) for i in range(self.n_steps)]

    def modes(self):
        return [self.step_mode[i] for i in range(self.n_steps)]

    def as_dict(self):
        return {
            "t": self.t, "k": self.k, "root": self.root, "children": self.children(),
            "steps": self.steps(), "modes": self.modes(), "batch": self.batch,
            "interleave": self.interleave, "arena_bytes": int(self.arena_bytes),
            "spmm_updates": self.spmm_updates, "ema_updates": self.ema_updates,
            "lemma1_ops": self.lemma1_ops, "exec_updates": self.exec_updates,
            "compulsory_bytes": self.compulsory_bytes, "automorphisms": self.automorphisms,
        }


class KernelStat(ctypes.Structure):
    _fields_ = [
        ("name", ctypes.c_char * 32), ("launches", ctypes.c_int32), ("total_ms", ctypes.c_double),
        ("alg_bytes", ctypes.c_double), ("updates", ctypes.c_double), ("layout_bytes", ctypes.c_double),
    ]


class Launch(ctypes.Structure):
    _fields_ = [
        ("kernel", ctypes.c_char * 96), ("family", ctypes.c_char * 16), ("step", ctypes.c_int32),
        ("h", ctypes.c_int32), ("a", ctypes.c_int32), ("p", ctypes.c_int32), ("colorings", ctypes.c_int32),
        ("ms", ctypes.c_double), ("alg_bytes", ctypes.c_double), ("layout_bytes", ctypes.c_double),
        ("updates", ctypes.c_double),
    ]


OPTION_DEFAULTS = {SC_OPT_MAX_BATCH: 64, SC_OPT_GRAPH: 0, SC_OPT_SEGMENT: 0, SC_OPT_REORDER: 1,
                   SC_OPT_INTERLEAVE: 0, SC_OPT_LDS_MAX: 0, SC_OPT_WAVE_ROW_MAX: -1, SC_OPT_CHAIN: 1}


class Job(ctypes.Structure):
    _fields_ = [
        ("graph_id", ctypes.c_int32), ("tmpl_id", ctypes.c_int32), ("k", ctypes.c_int32),
        ("seed", ctypes.c_uint64), ("first_coloring", ctypes.c_uint64), ("n_colorings", ctypes.c_int32),
        ("counts", ctypes.POINTER(ctypes.c_uint64)), ("overflow", ctypes.POINTER(ctypes.c_uint8)),
        ("est_maps", ctypes.c_double), ("est_copies", ctypes.c_double), ("status", ctypes.c_int32),
    ]


class Tune(ctypes.Structure):
    _fields_ = [("interleave", ctypes.c_int32), ("lds_max", ctypes.c_int32),
                ("batch", ctypes.c_int32), ("trials", ctypes.c_int32), ("ms", ctypes.c_double),
                ("seg", ctypes.c_int32), ("wave_row_max", ctypes.c_int32)]


class Estimate(ctypes.Structure):
    _fields_ = [("est_maps", ctypes.c_double), ("est_copies", ctypes.c_double),
                ("mean_maps", ctypes.c_double), ("rel_stderr", ctypes.c_double),
                ("colorings", ctypes.c_int64), ("per_group", ctypes.c_int64), ("needed", ctypes.c_int64),
                ("groups", ctypes.c_int32), ("exact", ctypes.c_int32)]


SC_EST_BOUND, SC_EST_SAMPLE = 0, 1
SC_ABL_FASCIA, SC_ABL_PFASCIA = 1, 2


class ServeCfg(ctypes.Structure):
    _fields_ = [("mem_budget_bytes", ctypes.c_uint64), ("max_inflight", ctypes.c_int32),
                ("max_batch", ctypes.c_int32)]


class Query(ctypes.Structure):
    _fields_ = [("graph_id", ctypes.c_int32), ("tmpl_id", ctypes.c_int32), ("k", ctypes.c_int32),
                ("seed", ctypes.c_uint64), ("first_coloring", ctypes.c_uint64),
                ("n_colorings", ctypes.c_int32)]


class Result(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("n_colorings", ctypes.c_int32),
                ("counts", ctypes.POINTER(ctypes.c_uint64)), ("overflow", ctypes.POINTER(ctypes.c_uint8)),
                ("est_maps", ctypes.c_double), ("est_copies", ctypes.c_double),
                ("submit_s", ctypes.c_double), ("start_s", ctypes.c_double), ("done_s", ctypes.c_double)]


class ServeStats(ctypes.Structure):
    _fields_ = [("passes", ctypes.c_uint64), ("colorings", ctypes.c_uint64), ("waiting", ctypes.c_int32),
                ("inflight", ctypes.c_int32), ("mem_bytes", ctypes.c_uint64),
                ("peak_mem_bytes", ctypes.c_uint64)]


class ScError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"libsc error {code}: {msg}")
        self.code = code


def lib():
    """Load libsc.so; raises if it has not been built.

    PyTorch is imported first: its wheel carries its own HIP runtime
    (libamdhip64.so.7, libhsa-runtime64.so.1), and loading it first lets
    libsc's dependencies resolve to those same, already loaded, libraries, so
    the process has one HIP runtime and the memory PyTorch's allocator hands
    the library belongs to the runtime that launches its kernels."""
    global _lib
    if _lib is None:
        if not os.path.exists(lib_path):
            raise RuntimeError(f"{lib_path} is missing: build it with `python -c 'import __graft_entry__ as g; g.build()'`")
        import torch  # noqa: F401  (see above: one HIP runtime per process)
        L = ctypes.CDLL(lib_path)
        sig = {
            "sc_create": (ctypes.c_int, [ctypes.c_int, ALLOC_FN, FREE_FN, _vp, ctypes.c_uint64, ctypes.POINTER(_vp)]),
            "sc_destroy": (ctypes.c_int, [_vp]),
            "sc_last_error": (ctypes.c_char_p, [_vp]),
            "sc_version": (ctypes.c_char_p, []),
            "sc_load_graph_csr": (ctypes.c_int, [_vp, ctypes.c_int64, ctypes.c_int64, _i64p, _i32p, _i32p]),
            "sc_unload_graph": (ctypes.c_int, [_vp, ctypes.c_int32]),
            "sc_load_template": (ctypes.c_int, [_vp, ctypes.c_int32, _i32p, ctypes.c_int32, _i32p]),
            "sc_load_template_plan": (ctypes.c_int, [_vp, ctypes.c_int32, ctypes.c_int32, _i32p, _i32p, _i32p]),
            "sc_set_colors": (ctypes.c_int, [_vp, ctypes.c_int32, ctypes.c_uint64]),
            "sc_plan_template": (ctypes.c_int, [ctypes.c_int32, _i32p, ctypes.c_int32, ctypes.c_int32,
                                                ctypes.c_int64, ctypes.c_int64, ctypes.c_int32,
                                                ctypes.POINTER(PlanInfo)]),
            "sc_plan_info": (ctypes.c_int, [_vp, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                            ctypes.POINTER(PlanInfo)]),
            "sc_colorset_rank": (ctypes.c_int64, [ctypes.c_uint32]),
            "sc_color_of": (ctypes.c_int32, [ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint64, ctypes.c_int32]),
            "sc_run": (ctypes.c_int, [_vp, ctypes.c_int32, ctypes.c_int32, ctypes.c_uint64, ctypes.c_int32,
                                      _vp, _u64p, _u8p, _dblp, _dblp]),
            "sc_run_static": (ctypes.c_int, [_vp, ctypes.c_int32, ctypes.c_int32, ctypes.c_uint64, ctypes.c_int32,
                                             _vp, _u64p, _u8p, _dblp, _dblp]),
            "sc_run_exact": (ctypes.c_int, [_vp, ctypes.c_int32, ctypes.c_int32, ctypes.c_uint64, ctypes.c_int32,
                                            _vp, _u64p, _u8p, _dblp, _dblp, _dblp]),
            "sc_run_mod": (ctypes.c_int, [_vp, ctypes.c_int32, ctypes.c_int32, ctypes.c_uint64, ctypes.c_int32,
                                          _vp, ctypes.c_uint64, _u64p]),
            "sc_hom_count": (ctypes.c_int, [_vp, ctypes.c_int32, ctypes.c_int32, _vp, _dblp]),
            "sc_run_ablation": (ctypes.c_int, [_vp, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_uint64,
                                               ctypes.c_int32, _vp, _u64p, _u8p]),
            "sc_colorings_for": (ctypes.c_int, [ctypes.c_int32, ctypes.c_int32, ctypes.c_double, ctypes.c_double,
                                                _i32p, _i64p]),
            "sc_estimate": (ctypes.c_int, [_vp, ctypes.c_int32, ctypes.c_int32, ctypes.c_uint64, ctypes.c_double,
                                           ctypes.c_double, ctypes.c_int32, ctypes.c_int64, _vp,
                                           ctypes.POINTER(Estimate)]),
            "sc_set_option": (ctypes.c_int, [_vp, ctypes.c_int32, ctypes.c_int64]),
            "sc_get_option": (ctypes.c_int, [_vp, ctypes.c_int32, _i64p]),
            "sc_run_batch": (ctypes.c_int, [_vp, ctypes.POINTER(Job), ctypes.c_int32, _vp]),
            "sc_autotune": (ctypes.c_int, [_vp, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                           ctypes.POINTER(Tune)]),
            "sc_tune_save": (ctypes.c_int, [_vp, ctypes.c_char_p]),
            "sc_tune_load": (ctypes.c_int, [_vp, ctypes.c_char_p, _i32p]),
            "sc_serve_start": (ctypes.c_int, [_vp, ctypes.POINTER(ServeCfg)]),
            "sc_submit": (ctypes.c_int, [_vp, ctypes.POINTER(Query), ctypes.POINTER(ctypes.c_uint64)]),
            "sc_poll": (ctypes.c_int, [_vp, ctypes.c_uint64, ctypes.POINTER(Result)]),
            "sc_serve_stats": (ctypes.c_int, [_vp, ctypes.POINTER(ServeStats)]),
            "sc_serve_stop": (ctypes.c_int, [_vp]),
            "sc_profile": (ctypes.c_int, [_vp, ctypes.c_int32]),
            "sc_profile_read": (ctypes.c_int, [_vp, ctypes.POINTER(KernelStat), ctypes.c_int32,
                                               _i32p]),
            "sc_valu_probe": (ctypes.c_int, [_vp, ctypes.c_int32, _vp, _dblp]),
            "sc_profile_launches": (ctypes.c_int, [_vp, ctypes.POINTER(Launch), ctypes.c_int32, _i32p]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _p(a, t):
    return a.ctypes.data_as(t)


def sc_version() -> str:
    return lib().sc_version().decode()


def colorings_for(k, t, eps, delta):
    """(groups, per_group) of the (eps, delta) median-of-means bound; pure host."""
    m, g = ctypes.c_int32(), ctypes.c_int64()
    rc = lib().sc_colorings_for(k, t, eps, delta, ctypes.byref(m), ctypes.byref(g))
    if rc:
        raise ScError(rc, f"sc_colorings_for(k={k}, t={t}, eps={eps}, delta={delta}) rejected")
    return m.value, g.value


def _edges_array(t, edges):
    e = np.asarray(edges, dtype=np.int32).reshape(-1)
    if e.size != 2 * (t - 1):
        raise ValueError("need t-1 edges")
    return np.ascontiguousarray(e if e.size else np.zeros(2, np.int32))


def sc_plan_template(t, edges, root, k, n, nnz, batch=1) -> PlanInfo:
    """Host-only planning (no device needed)."""
    out = PlanInfo()
    e = _edges_array(t, edges)
    rc = lib().sc_plan_template(t, _p(e, _i32p), root, k, n, nnz, batch, ctypes.byref(out))
    if rc:
        raise ScError(rc, "sc_plan_template failed")
    return out


def sc_colorset_rank(mask: int) -> int:
    return int(lib().sc_colorset_rank(mask))


def sc_color_of(seed: int, coloring: int, vertex: int, k: int) -> int:
    return int(lib().sc_color_of(seed & (2**64 - 1), coloring, vertex, k))


class Context:
    """One libsc context on a HIP device.

    Device memory comes from PyTorch's caching allocator (the library's
    required allocator hook), so the library's tables show in
    ``torch.cuda.memory_allocated()``; every call that takes a stream runs on
    PyTorch's current stream unless given another (a ``torch.cuda.Stream`` or
    a raw hipStream_t as an int).  PyTorch's default stream is the null
    stream, for which the library uses its own non-blocking stream."""

    def __init__(self, device: int = 0, budget: int = 0):
        import torch
        L = lib()
        dev = int(device)

        def _alloc(nbytes, stream, user):
            try:
                return int(torch.cuda.caching_allocator_alloc(int(nbytes), dev, stream or 0))
            except Exception:
                return None

        def _free(ptr, nbytes, stream, user):
            try:
                torch.cuda.caching_allocator_delete(ptr)
            except Exception:
                pass

        self._cbs = (ALLOC_FN(_alloc), FREE_FN(_free))
        self._device = dev
        self._torch = torch
        h = _vp()
        rc = L.sc_create(dev, self._cbs[0], self._cbs[1], None, budget, ctypes.byref(h))
        if rc:
            raise ScError(rc, "sc_create failed (no usable HIP device?)")
        self._h = h
        self._L = L

    def _stream(self, stream):
        """hipStream_t for a call: PyTorch's current stream unless given."""
        if stream is None:
            return self._torch.cuda.current_stream(self._device).cuda_stream or None
        if isinstance(stream, int):
            return stream or None
        return stream.cuda_stream or None

    # -- plumbing
    def _check(self, rc):
        if rc:
            raise ScError(rc, self._L.sc_last_error(self._h).decode())

    def close(self):
        if getattr(self, "_h", None):
            self._L.sc_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    # -- API
    def last_error(self) -> str:
        return self._L.sc_last_error(self._h).decode()

    def load_graph_csr(self, n, row_ptr, col_idx) -> int:
        rp = np.ascontiguousarray(row_ptr, dtype=np.int64)
        ci = np.ascontiguousarray(col_idx, dtype=np.int32)
        nnz = int(rp[-1]) if rp.size else 0
        if ci.size == 0:
            ci = np.zeros(1, np.int32)
        gid = ctypes.c_int32()
        self._check(self._L.sc_load_graph_csr(self._h, n, nnz, _p(rp, _i64p), _p(ci, _i32p), ctypes.byref(gid)))
        return gid.value

    def load_graph(self, g) -> int:
        return self.load_graph_csr(g.n, g.row_ptr, g.col_idx)

    def unload_graph(self, gid: int):
        self._check(self._L.sc_unload_graph(self._h, gid))

    def load_template(self, t, edges, root=-1) -> int:
        e = _edges_array(t, edges)
        tid = ctypes.c_int32()
        self._check(self._L.sc_load_template(self._h, t, _p(e, _i32p), root, ctypes.byref(tid)))
        return tid.value

    def load_template_plan(self, t, root, children) -> int:
        ptr = np.zeros(t + 1, np.int32)
        idx = []
        for u in range(t):
            idx.extend(children[u])
            ptr[u + 1] = len(idx)
        ci = np.asarray(idx if idx else [0], np.int32)
        tid = ctypes.c_int32()
        self._check(self._L.sc_load_template_plan(self._h, t, root, _p(ptr, _i32p), _p(ci, _i32p), ctypes.byref(tid)))
        return tid.value

    def set_colors(self, k, seed):
        self._check(self._L.sc_set_colors(self._h, k, seed & (2**64 - 1)))

    def set_option(self, opt, value):
        self._check(self._L.sc_set_option(self._h, opt, int(value)))

    def get_option(self, opt) -> int:
        v = ctypes.c_int64()
        self._check(self._L.sc_get_option(self._h, opt, ctypes.byref(v)))
        return v.value

    def profile(self, enable: bool):
        self._check(self._L.sc_profile(self._h, 1 if enable else 0))

    def profile_read(self):
        """{family: {launches, total_ms, alg_bytes, updates}} of the recorded launches."""
        cap = 64
        arr = (KernelStat * cap)()
        n = ctypes.c_int32()
        self._check(self._L.sc_profile_read(self._h, arr, cap, ctypes.byref(n)))
        return {arr[i].name.decode(): {"launches": arr[i].launches, "total_ms": arr[i].total_ms,
                                       "alg_bytes": arr[i].alg_bytes, "layout_bytes": arr[i].layout_bytes,
                                       "updates": arr[i].updates}
                for i in range(min(n.value, cap))}

    def valu_probe(self, form=0, stream=None):
        """Exact 64-bit multiply-adds per second of the device's vector ALU
        (form 0: 128-bit product, 1: three 32-bit multiplies, 2: 32-bit second
        operand)."""
        out = ctypes.c_double()
        self._check(self._L.sc_valu_probe(self._h, int(form), self._stream(stream), ctypes.byref(out)))
        return out.value

    def profile_launches(self):
        """Every recorded launch in order, as dicts (kernel, family, step, h, a, p,
        colorings, ms, alg_bytes, layout_bytes, updates)."""
        n = ctypes.c_int32()
        self._check(self._L.sc_profile_launches(self._h, None, 0, ctypes.byref(n)))
        arr = (Launch * max(1, n.value))()
        self._check(self._L.sc_profile_launches(self._h, arr, n.value, ctypes.byref(n)))
        out = []
        for r in arr[:n.value]:
            d = {f: getattr(r, f) for f, _ in Launch._fields_}
            d["kernel"], d["family"] = r.kernel.decode(), r.family.decode()
            out.append(d)
        return out

    def plan_info(self, gid, tid, n_colorings=1) -> PlanInfo:
        out = PlanInfo()
        self._check(self._L.sc_plan_info(self._h, gid, tid, n_colorings, ctypes.byref(out)))
        return out

    def run_batch(self, jobs, stream=None):
        """jobs: list of dicts {graph_id, tmpl_id, k, seed, first, n}.  Returns a
        list of (counts, overflow, est_maps, est_copies, status) per job."""
        arr = (Job * max(1, len(jobs)))()
        bufs = []
        for i, j in enumerate(jobs):
            n = int(j["n"])
            cnt = np.zeros(max(n, 1), np.uint64)
            ovf = np.zeros(max(n, 1), np.uint8)
            bufs.append((cnt, ovf, n))
            arr[i].graph_id, arr[i].tmpl_id, arr[i].k = j["graph_id"], j["tmpl_id"], j["k"]
            arr[i].seed = j["seed"] & (2**64 - 1)
            arr[i].first_coloring = j.get("first", 0)
            arr[i].n_colorings = n
            arr[i].counts = _p(cnt, _u64p)
            arr[i].overflow = _p(ovf, _u8p)
        rc = self._L.sc_run_batch(self._h, arr, len(jobs), self._stream(stream))
        out = [(bufs[i][0][:bufs[i][2]], bufs[i][1][:bufs[i][2]], arr[i].est_maps, arr[i].est_copies,
                arr[i].status) for i in range(len(jobs))]
        if rc and all(o[4] == 0 for o in out):
            self._check(rc)
        return out

    def autotune(self, gid, tid, n_colorings):
        t = Tune()
        self._check(self._L.sc_autotune(self._h, gid, tid, n_colorings, ctypes.byref(t)))
        return {"interleave": t.interleave, "lds_max": t.lds_max, "seg": t.seg, "wave_row_max": t.wave_row_max,
                "batch": t.batch, "trials": t.trials, "ms": t.ms}

    def tune_save(self, path):
        self._check(self._L.sc_tune_save(self._h, str(path).encode()))

    def tune_load(self, path):
        n = ctypes.c_int32()
        self._check(self._L.sc_tune_load(self._h, str(path).encode(), ctypes.byref(n)))
        return n.value

    # -- serving
    def serve_start(self, mem_budget_bytes=0, max_inflight=4, max_batch=64):
        cfg = ServeCfg(mem_budget_bytes, max_inflight, max_batch)
        self._check(self._L.sc_serve_start(self._h, ctypes.byref(cfg)))

    def submit(self, gid, tid, k, seed, first, n_colorings) -> int:
        q = Query(gid, tid, k, seed & (2**64 - 1), first, n_colorings)
        t = ctypes.c_uint64()
        self._check(self._L.sc_submit(self._h, ctypes.byref(q), ctypes.byref(t)))
        return t.value

    def poll(self, ticket, n_colorings):
        """None while the query runs; else a dict with counts, overflow,
        estimates, status and timestamps."""
        cnt = np.zeros(max(n_colorings, 1), np.uint64)
        ovf = np.zeros(max(n_colorings, 1), np.uint8)
        r = Result()
        r.counts = _p(cnt, _u64p)
        r.overflow = _p(ovf, _u8p)
        rc = self._L.sc_poll(self._h, ticket, ctypes.byref(r))
        if rc == SC_EBUSY:
            return None
        self._check(rc)
        return {"status": r.status, "counts": cnt[:n_colorings], "overflow": ovf[:n_colorings],
                "est_maps": r.est_maps, "est_copies": r.est_copies, "submit_s": r.submit_s,
                "start_s": r.start_s, "done_s": r.done_s}

    def serve_stats(self):
        st = ServeStats()
        self._check(self._L.sc_serve_stats(self._h, ctypes.byref(st)))
        return {f: getattr(st, f) for f, _ in ServeStats._fields_}

    def serve_stop(self):
        self._check(self._L.sc_serve_stop(self._h))

    def run(self, gid, tid, first, n_colorings, stream=None):
        """Returns (counts uint64[R], overflow uint8[R], est_maps, est_copies)."""
        R = int(n_colorings)
        counts = np.zeros(max(R, 1), np.uint64)
        ovf = np.zeros(max(R, 1), np.uint8)
        em, ec = ctypes.c_double(), ctypes.c_double()
        self._check(self._L.sc_run(self._h, gid, tid, first, R, self._stream(stream), _p(counts, _u64p), _p(ovf, _u8p),
                                   ctypes.byref(em), ctypes.byref(ec)))
        return counts[:R], ovf[:R], em.value, ec.value

    def run_static(self, gid, tid, first, n_colorings, stream=None):
        """As run(), through the allocation-free entry point (every buffer in the
        library's per-device static array of SC_STATIC_SCRATCH_BYTES)."""
        R = int(n_colorings)
        counts = np.zeros(max(R, 1), np.uint64)
        ovf = np.zeros(max(R, 1), np.uint8)
        em, ec = ctypes.c_double(), ctypes.c_double()
        self._check(self._L.sc_run_static(self._h, gid, tid, first, R, self._stream(stream), _p(counts, _u64p),
                                          _p(ovf, _u8p), ctypes.byref(em), ctypes.byref(ec)))
        return counts[:R], ovf[:R], em.value, ec.value

    def run_exact(self, gid, tid, first, n_colorings, stream=None):
        """Returns (counts [int], exact uint8[R], hom_bound, est_maps, est_copies): the
        counts as Python integers, combined from four uint64 limbs."""
        R = int(n_colorings)
        limbs = np.zeros((max(R, 1), 4), np.uint64)
        exact = np.zeros(max(R, 1), np.uint8)
        hb, em, ec = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
        self._check(self._L.sc_run_exact(self._h, gid, tid, first, R, self._stream(stream), _p(limbs, _u64p), _p(exact, _u8p),
                                         ctypes.byref(hb), ctypes.byref(em), ctypes.byref(ec)))
        counts = [sum(int(limbs[r, i]) << (64 * i) for i in range(4)) for r in range(R)]
        return counts, exact[:R], hb.value, em.value, ec.value

    def run_mod(self, gid, tid, first, n_colorings, p, stream=None):
        """Returns uint64[R]: each colouring's count mod p."""
        R = int(n_colorings)
        res = np.zeros(max(R, 1), np.uint64)
        self._check(self._L.sc_run_mod(self._h, gid, tid, first, R, self._stream(stream), int(p), _p(res, _u64p)))
        return res[:R]

    def run_ablation(self, gid, tid, variant, first, n_colorings, stream=None):
        """Counts by the FASCIA or PFASCIA baseline kernels: (counts uint64[R], overflow uint8[R])."""
        R = int(n_colorings)
        counts = np.zeros(max(R, 1), np.uint64)
        ovf = np.zeros(max(R, 1), np.uint8)
        self._check(self._L.sc_run_ablation(self._h, gid, tid, variant, first, R, self._stream(stream), _p(counts, _u64p),
                                            _p(ovf, _u8p)))
        return counts[:R], ovf[:R]

    def estimate(self, gid, tid, eps, delta, mode=SC_EST_BOUND, max_colorings=0, first=0, stream=None):
        """(eps, delta) estimate by the median of means; returns an Estimate."""
        out = Estimate()
        self._check(self._L.sc_estimate(self._h, gid, tid, first, eps, delta, mode, max_colorings, self._stream(stream),
                                        ctypes.byref(out)))
        return out

    def hom_count(self, gid, tid, stream=None):
        """Homomorphisms of the template into the graph (double)."""
        out = ctypes.c_double()
        self._check(self._L.sc_hom_count(self._h, gid, tid, self._stream(stream), ctypes.byref(out)))
        return out.value
