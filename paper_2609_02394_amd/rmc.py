"""ctypes binding of librmc (include/rmc.h). Argument marshalling only: every step
of the method runs in the library's HIP kernels. PyTorch provides the device
arena and the stream.

Importing this module loads ``librmc.so`` from the package directory and fails
loudly if it is missing (build it with ``python -m paper_2609_02394_amd.build``).
"""
from __future__ import annotations

import ctypes as C
import os
from typing import List, Optional, Sequence, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "librmc.so")

OK, ERR_ARG, ERR_OOM, ERR_NOCONV, ERR_HIP, ERR_STATE = range(6)
FP64, FP32, BF16 = 0, 1, 2
OPS = {"X": 1, "T": 2, "Z": 3}
STATUS_NAMES = {0: "OK", 1: "ERR_ARG", 2: "ERR_OOM", 3: "ERR_NOCONV", 4: "ERR_HIP", 5: "ERR_STATE"}

EXPORTED = (
    "rmc_default_opts", "rmc_create", "rmc_destroy", "rmc_last_error", "rmc_arena_usage",
    "rmc_module_ed", "rmc_project_ops", "rmc_couple_solve", "rmc_recurse", "rmc_recurse_chain",
    "rmc_recurse_batch",
    "rmc_module_info", "rmc_module_basis", "rmc_module_op", "rmc_module_free", "rmc_module_lift",
    "rmc_leaf_hamiltonian", "rmc_kron_apply", "rmc_sym_eig", "rmc_module_import",
    "rmc_profile", "rmc_profile_read", "rmc_profile_read_precision",
    "rmc_serve_start", "rmc_submit", "rmc_poll", "rmc_serve_stop", "rmc_merge_bound",
    "rmc_profile_read_kernel", "rmc_kron_apply_noalloc",
)
PROF_KRON_STEP, PROF_KRON_FILTER, PROF_PAULI = 0, 1, 2


class Term(C.Structure):
    _fields_ = [("coef", C.c_double), ("nsite", C.c_int), ("site", C.c_int * 2), ("op", C.c_int * 2)]


class LeafDesc(C.Structure):
    _fields_ = [("n_sites", C.c_int), ("n_terms", C.c_int), ("terms", C.POINTER(Term))]


class BondDesc(C.Structure):
    _fields_ = [("n_terms", C.c_int), ("coef", C.POINTER(C.c_double)),
                ("opA", C.POINTER(C.c_int)), ("opB", C.POINTER(C.c_int))]


class ChainDesc(C.Structure):
    _fields_ = [("n_sites", C.c_int), ("leaf_sites", C.c_int), ("n_terms", C.c_int),
                ("terms", C.POINTER(Term)), ("k", C.c_int), ("q", C.c_int)]


class TreeNode(C.Structure):
    _fields_ = [("left", C.c_int), ("right", C.c_int), ("n_sites", C.c_int), ("n_terms", C.c_int),
                ("terms", C.POINTER(Term)), ("k", C.c_int)]


class TreeDesc(C.Structure):
    _fields_ = [("n_nodes", C.c_int), ("nodes", C.POINTER(TreeNode)), ("k", C.c_int), ("q", C.c_int)]


class JobDesc(C.Structure):
    _fields_ = [("tree", C.POINTER(TreeDesc)), ("chain", C.POINTER(ChainDesc))]


class SolveOpts(C.Structure):
    _fields_ = [("precision", C.c_int), ("tol", C.c_double), ("gap_tol", C.c_double),
                ("max_iter", C.c_int), ("guard", C.c_int), ("max_degree", C.c_int),
                ("seed", C.c_ulonglong)]


class LevelReport(C.Structure):
    _fields_ = [("level", C.c_int), ("width", C.c_int), ("kind", C.c_int), ("k_req", C.c_int),
                ("k_eff", C.c_int), ("iters", C.c_int), ("matvecs", C.c_int), ("reused", C.c_int),
                ("rr_sweeps", C.c_int), ("gap", C.c_double), ("max_res", C.c_double), ("ms", C.c_double)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class Report(C.Structure):
    _fields_ = [("capacity", C.c_int), ("n_records", C.c_int), ("records", C.POINTER(LevelReport)),
                ("n_leaf_ed", C.c_int), ("n_merges", C.c_int), ("total_ms", C.c_double)]


def load_library(path: str = LIB_PATH) -> C.CDLL:
    if not os.path.exists(path):
        raise RuntimeError(f"librmc.so not built ({path}); run python -m paper_2609_02394_amd.build")
    lib = C.CDLL(path)
    vp, i, d, sz = C.c_void_p, C.c_int, C.c_double, C.c_size_t
    P = C.POINTER
    sig = {
        "rmc_default_opts": (None, [P(SolveOpts)]),
        "rmc_create": (i, [P(vp), i, vp, sz, vp]),
        "rmc_destroy": (i, [vp]),
        "rmc_last_error": (C.c_char_p, [vp]),
        "rmc_arena_usage": (i, [vp, P(sz), P(sz)]),
        "rmc_module_ed": (i, [vp, P(LeafDesc), i, P(SolveOpts), P(vp)]),
        "rmc_project_ops": (i, [vp, vp, i, P(i), P(i), P(i)]),
        "rmc_couple_solve": (i, [vp, vp, vp, P(BondDesc), i, i, P(SolveOpts), P(vp), P(d),
                                 P(LevelReport)]),
        "rmc_recurse": (i, [vp, P(TreeDesc), P(SolveOpts), P(d), P(Report)]),
        "rmc_recurse_chain": (i, [vp, P(ChainDesc), P(SolveOpts), P(d), P(Report)]),
        "rmc_recurse_batch": (i, [vp, i, P(JobDesc), P(SolveOpts), P(d), i, P(i)]),
        "rmc_module_info": (i, [vp, P(i), P(i), P(i), P(d)]),
        "rmc_module_basis": (i, [vp, vp, P(d)]),
        "rmc_module_lift": (i, [vp, vp, vp]),
        "rmc_module_op": (i, [vp, vp, i, P(d)]),
        "rmc_module_free": (i, [vp, vp]),
        "rmc_leaf_hamiltonian": (i, [vp, P(LeafDesc), vp]),
        "rmc_kron_apply": (i, [vp, vp, vp, P(BondDesc), i, i, vp, vp]),
        "rmc_kron_apply_noalloc": (i, [vp, vp, vp, P(BondDesc), i, i, vp, vp]),
        "rmc_sym_eig": (i, [vp, i, i, vp, vp, vp]),
        "rmc_module_import": (i, [vp, i, i, i, P(d), P(d), i, P(i), P(i), P(d), P(vp)]),
        "rmc_profile": (i, [vp, i]),
        "rmc_profile_read": (i, [vp, P(C.c_longlong), P(d), P(d), P(d)]),
        "rmc_profile_read_precision": (i, [vp, i, P(C.c_longlong), P(d), P(d), P(d)]),
        "rmc_profile_read_kernel": (i, [vp, i, i, P(C.c_longlong), P(d), P(d), P(d)]),
        "rmc_serve_start": (i, [vp, P(SolveOpts), i, sz]),
        "rmc_submit": (i, [vp, P(JobDesc), P(C.c_ulonglong)]),
        "rmc_poll": (i, [vp, C.c_ulonglong, P(i), P(d), i, P(i), P(d)]),
        "rmc_serve_stop": (i, [vp]),
        "rmc_merge_bound": (i, [vp, vp, P(LeafDesc), vp, P(LeafDesc), P(BondDesc), P(SolveOpts),
                                P(d)]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    return lib


_lib: Optional[C.CDLL] = None


def lib() -> C.CDLL:
    global _lib
    if _lib is None:
        _lib = load_library()
    return _lib


class RmcError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


def make_terms(terms) -> "C.Array":
    """terms: iterable of (coef, ((site, op), ...)) with op a letter or an int."""
    terms = list(terms)
    arr = (Term * max(1, len(terms)))()
    for t, (c, ops) in enumerate(terms):
        arr[t].coef = float(c)
        arr[t].nsite = len(ops)
        for u, (s, o) in enumerate(ops):
            arr[t].site[u] = int(s)
            arr[t].op[u] = OPS[o] if isinstance(o, str) else int(o)
    return arr, len(terms)


def make_tree(nodes, k: int, q: int):
    """A TreeDesc from nodes (children before parents, the last the root):
    ("leaf", n_sites, terms, k_node) with terms as for make_terms (local sites), or
    ("merge", left, right, terms, k_node) with terms (coef, site_A, op_A, site_B, op_B).
    Returns (desc, keep-alive list)."""
    arr = (TreeNode * max(1, len(nodes)))()
    keep = [arr]
    for i, nd in enumerate(nodes):
        if nd[0] == "leaf":
            _, n, terms, kn = nd
            t, nt = make_terms(terms)
            arr[i] = TreeNode(-1, -1, int(n), nt, t, int(kn))
        else:
            _, l, r, terms, kn = nd
            t, nt = make_terms([(c, ((sa, oa), (sb, ob))) for c, sa, oa, sb, ob in terms])
            arr[i] = TreeNode(int(l), int(r), 0, nt, t, int(kn))
        keep.append(t)
    desc = TreeDesc(len(nodes), arr, int(k), int(q))
    keep.append(desc)
    return desc, keep


def make_job(job):
    """A JobDesc from a chain tuple (n_sites, leaf_sites, terms, k, q) or a tree tuple
    ("tree", nodes, k, q). Returns (desc, q, keep-alive list)."""
    if job[0] == "tree":
        _, nodes, k, q = job
        td, keep = make_tree(nodes, k, q)
        jd = JobDesc(C.pointer(td), None)
        return jd, q, keep + [td]
    ns, ls, terms, k, q = job
    arr, nt = make_terms(terms)
    cd = ChainDesc(ns, ls, nt, arr, int(k), int(q))
    return JobDesc(None, C.pointer(cd)), q, [arr, cd]


class JobBatch:
    """Jobs marshalled once into the library's job descriptors, for callers that solve
    the same batch repeatedly (the descriptors are read-only inputs of
    rmc_recurse_batch and stay valid while this object lives)."""

    def __init__(self, jobs):
        self.n = len(jobs)
        self.descs = (JobDesc * max(1, self.n))()
        self.keep = []
        self.qmax = 1
        for j, job in enumerate(jobs):
            jd, q, kp = make_job(job)
            self.descs[j] = jd
            self.keep.append(kp)
            self.qmax = max(self.qmax, q)

    def __len__(self):
        return self.n


def default_opts(**kw) -> SolveOpts:
    o = SolveOpts()
    lib().rmc_default_opts(C.byref(o))
    for k, v in kw.items():
        setattr(o, k, v)
    return o


class Module:
    def __init__(self, ctx: "Context", handle):
        self.ctx = ctx
        self.h = handle

    def info(self):
        k, dim, ns = C.c_int(), C.c_int(), C.c_int()
        self.ctx._check(lib().rmc_module_info(self.h, C.byref(k), C.byref(dim), C.byref(ns), None))
        E = np.zeros(max(1, k.value))
        self.ctx._check(lib().rmc_module_info(self.h, None, None, None,
                                              E.ctypes.data_as(C.POINTER(C.c_double))))
        return {"k_eff": k.value, "dim": dim.value, "n_sites": ns.value, "E": E[: k.value]}

    def basis(self) -> np.ndarray:
        inf = self.info()
        out = np.zeros((inf["k_eff"], inf["dim"]))
        self.ctx._check(lib().rmc_module_basis(self.ctx.h, self.h,
                                               out.ctypes.data_as(C.POINTER(C.c_double))))
        return out

    def lift(self):
        """Retained states as full-space vectors: device tensor (k_eff, 2**n_sites)."""
        import torch

        inf = self.info()
        out = torch.empty((inf["k_eff"], 1 << inf["n_sites"]), dtype=torch.float64,
                          device=f"cuda:{self.ctx.device}")
        self.ctx._check(lib().rmc_module_lift(self.ctx.h, self.h, C.c_void_p(out.data_ptr())))
        return out

    def op(self, op_id: int) -> np.ndarray:
        k = self.info()["k_eff"]
        out = np.zeros((k, k))
        self.ctx._check(lib().rmc_module_op(self.ctx.h, self.h, int(op_id),
                                            out.ctypes.data_as(C.POINTER(C.c_double))))
        return out

    def project_ops(self, sites: Sequence[int], ops: Sequence) -> List[int]:
        n = len(sites)
        s = (C.c_int * max(1, n))(*[int(x) for x in sites])
        o = (C.c_int * max(1, n))(*[OPS[x] if isinstance(x, str) else int(x) for x in ops])
        ids = (C.c_int * max(1, n))()
        self.ctx._check(lib().rmc_project_ops(self.ctx.h, self.h, n, s, o, ids))
        return list(ids)[:n]

    def free(self):
        if self.h:
            self.ctx._check(lib().rmc_module_free(self.ctx.h, self.h))
            self.h = None


def _bond(coefs, opA, opB):
    n = len(coefs)
    c = (C.c_double * max(1, n))(*[float(x) for x in coefs])
    a = (C.c_int * max(1, n))(*[int(x) for x in opA])
    b = (C.c_int * max(1, n))(*[int(x) for x in opB])
    bd = BondDesc(n, c, a, b)
    return bd, (c, a, b)


class Context:
    """One librmc context on one GPU, with a torch-allocated device arena."""

    def __init__(self, arena_bytes: int = 2 << 30, device: int = 0, stream=None):
        import torch

        if not torch.cuda.is_available():
            raise RuntimeError("librmc needs a ROCm GPU")
        self.device = device
        self.arena = torch.empty(int(arena_bytes), dtype=torch.uint8, device=f"cuda:{device}")
        self.stream = stream if stream is not None else torch.cuda.current_stream(device)
        h = C.c_void_p()
        st = lib().rmc_create(C.byref(h), device, C.c_void_p(self.arena.data_ptr()),
                              int(arena_bytes), C.c_void_p(self.stream.cuda_stream))
        if st != OK:
            raise RmcError(st, "rmc_create failed")
        self.h = h

    def close(self):
        if getattr(self, "h", None):
            lib().rmc_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, st, allow=()):
        if st != OK and st not in allow:
            raise RmcError(st, lib().rmc_last_error(self.h).decode())
        return st

    def profile(self, enable: bool):
        self._check(lib().rmc_profile(self.h, int(bool(enable))))

    def profile_read(self, precision: Optional[int] = None, kernel: Optional[int] = None):
        """Launch totals since profile(True): all Kronecker launches, those of one
        precision (FP64 / FP32 / BF16), or those of one kernel kind (PROF_KRON_STEP,
        PROF_KRON_FILTER, PROF_PAULI) and precision."""
        n, f, b, ms = C.c_longlong(), C.c_double(), C.c_double(), C.c_double()
        if kernel is not None:
            self._check(lib().rmc_profile_read_kernel(self.h, int(kernel), int(precision or 0),
                                                      C.byref(n), C.byref(f), C.byref(b),
                                                      C.byref(ms)))
        elif precision is None:
            self._check(lib().rmc_profile_read(self.h, C.byref(n), C.byref(f), C.byref(b),
                                               C.byref(ms)))
        else:
            self._check(lib().rmc_profile_read_precision(self.h, int(precision), C.byref(n),
                                                         C.byref(f), C.byref(b), C.byref(ms)))
        return {"launches": n.value, "flops": f.value, "bytes": b.value, "ms": ms.value}

    def arena_usage(self) -> Tuple[int, int]:
        a, b = C.c_size_t(), C.c_size_t()
        self._check(lib().rmc_arena_usage(self.h, C.byref(a), C.byref(b)))
        return a.value, b.value

    # -- the four calls of the method -----------------------------------------
    def module_ed(self, n_sites: int, terms, k: int, opts: Optional[SolveOpts] = None) -> Module:
        arr, nt = make_terms(terms)
        ld = LeafDesc(n_sites, nt, arr)
        out = C.c_void_p()
        self._check(lib().rmc_module_ed(self.h, C.byref(ld), int(k),
                                        C.byref(opts) if opts else None, C.byref(out)))
        return Module(self, out)

    def module_import(self, n_sites: int, E, ops=(), basis=None, dim: Optional[int] = None) -> Module:
        """ops: list of (site, op, k x k array)."""
        E = np.ascontiguousarray(E, dtype=np.float64)
        k = len(E)
        if dim is None:
            dim = basis.shape[1] if basis is not None else k
        dp = C.POINTER(C.c_double)
        b = None
        if basis is not None:
            basis = np.ascontiguousarray(basis, dtype=np.float64)
            b = basis.ctypes.data_as(dp)
        n = len(ops)
        sites = (C.c_int * max(1, n))(*[int(s) for s, _, _ in ops])
        opc = (C.c_int * max(1, n))(*[OPS[o] if isinstance(o, str) else int(o) for _, o, _ in ops])
        data = np.ascontiguousarray(np.stack([np.asarray(m, dtype=np.float64) for _, _, m in ops])
                                    if n else np.zeros((1, k, k)))
        out = C.c_void_p()
        self._check(lib().rmc_module_import(self.h, int(n_sites), k, int(dim), E.ctypes.data_as(dp),
                                            b, n, sites, opc, data.ctypes.data_as(dp), C.byref(out)))
        return Module(self, out)

    def couple_solve(self, A: Module, B: Module, coefs, opA, opB, k_keep: int, q: int,
                     opts: Optional[SolveOpts] = None, want_module: bool = True):
        bd, keep = _bond(coefs, opA, opB)
        out = C.c_void_p()
        e = np.zeros(q)
        rep = LevelReport()
        st = lib().rmc_couple_solve(self.h, A.h, B.h, C.byref(bd), int(k_keep), int(q),
                                    C.byref(opts) if opts else None,
                                    C.byref(out) if want_module else None,
                                    e.ctypes.data_as(C.POINTER(C.c_double)), C.byref(rep))
        self._check(st)
        return (Module(self, out) if want_module else None), e, rep.as_dict()

    def merge_bound(self, A: Module, terms_A, B: Module, terms_B, coefs, opA, opB,
                    opts: Optional[SolveOpts] = None):
        """Single-merge diagnostics of two leaf modules built from terms_A / terms_B:
        dict with a, b, c, gamma, r, b2_over_gamma, E0."""
        arr_a, na = make_terms(terms_A)
        arr_b, nb = make_terms(terms_B)
        la = LeafDesc(A.info()["n_sites"], na, arr_a)
        lb = LeafDesc(B.info()["n_sites"], nb, arr_b)
        bd, keep = _bond(coefs, opA, opB)
        out = np.zeros(7)
        self._check(lib().rmc_merge_bound(self.h, A.h, C.byref(la), B.h, C.byref(lb), C.byref(bd),
                                          C.byref(opts) if opts else None,
                                          out.ctypes.data_as(C.POINTER(C.c_double))))
        return dict(zip(("a", "b", "c", "gamma", "r", "b2_over_gamma", "E0"), out.tolist()))

    def recurse(self, n_sites: int, leaf_sites: int, terms, k: int, q: int,
                opts: Optional[SolveOpts] = None, report_capacity: int = 64):
        """The recursion over a chain (rmc_recurse_chain)."""
        arr, nt = make_terms(terms)
        ch = ChainDesc(n_sites, leaf_sites, nt, arr, int(k), int(q))
        e = np.zeros(q)
        recs = (LevelReport * report_capacity)()
        rep = Report(report_capacity, 0, recs, 0, 0, 0.0)
        self._check(lib().rmc_recurse_chain(self.h, C.byref(ch), C.byref(opts) if opts else None,
                                            e.ctypes.data_as(C.POINTER(C.c_double)), C.byref(rep)))
        return e, self._report(rep, recs, report_capacity)

    def recurse_tree(self, nodes, k: int, q: int, opts: Optional[SolveOpts] = None,
                     report_capacity: int = 256, allow=()):
        """The recursion over a module tree (rmc_recurse); nodes as for make_tree.
        Returns (energies, report, status)."""
        td, keep = make_tree(nodes, k, q)
        e = np.full(q, np.nan)
        recs = (LevelReport * report_capacity)()
        rep = Report(report_capacity, 0, recs, 0, 0, 0.0)
        st = self._check(lib().rmc_recurse(self.h, C.byref(td), C.byref(opts) if opts else None,
                                           e.ctypes.data_as(C.POINTER(C.c_double)), C.byref(rep)),
                         allow=allow)
        return e, self._report(rep, recs, report_capacity), st

    @staticmethod
    def _report(rep, recs, cap):
        records = [recs[i].as_dict() for i in range(min(rep.n_records, cap))]
        return {"records": records, "n_leaf_ed": rep.n_leaf_ed, "n_merges": rep.n_merges,
                "total_ms": rep.total_ms}

    def recurse_batch(self, jobs, opts: Optional[SolveOpts] = None):
        """jobs: a JobBatch, or chain tuples (n_sites, leaf_sites, terms, k, q) and tree
        tuples ("tree", nodes, k, q). Returns energies (n, qmax), per-job status codes
        and the call's status."""
        b = jobs if isinstance(jobs, JobBatch) else JobBatch(jobs)
        n = b.n
        e = np.full((max(1, n), b.qmax), np.nan)
        sts = (C.c_int * max(1, n))()
        st = lib().rmc_recurse_batch(self.h, n, b.descs, C.byref(opts) if opts else None,
                                     e.ctypes.data_as(C.POINTER(C.c_double)), b.qmax, sts)
        return e[:n], list(sts)[:n], st

    # -- serving (continuous batching) --------------------------------------------
    def serve_start(self, opts: Optional[SolveOpts] = None, max_inflight: int = 64,
                    mem_budget: int = 0):
        self._check(lib().rmc_serve_start(self.h, C.byref(opts) if opts else None,
                                          int(max_inflight), int(mem_budget)))

    def submit(self, *job) -> int:
        """Queue a chain (n_sites, leaf_sites, terms, k, q) or a tree ("tree", nodes, k, q)."""
        jd, q, keep = make_job(job)
        jid = C.c_ulonglong()
        self._check(lib().rmc_submit(self.h, C.byref(jd), C.byref(jid)))
        return jid.value

    def poll(self, job_id: int, q: int):
        """(done, energies, status, latency_ms); energies (q of them) valid once done."""
        done, st, lat = C.c_int(), C.c_int(), C.c_double()
        e = np.full(q, np.nan)
        self._check(lib().rmc_poll(self.h, C.c_ulonglong(job_id), C.byref(done),
                                   e.ctypes.data_as(C.POINTER(C.c_double)), int(q), C.byref(st),
                                   C.byref(lat)))
        return bool(done.value), e, st.value, lat.value

    def serve_stop(self):
        self._check(lib().rmc_serve_stop(self.h))

    # -- kernel-level entry points ---------------------------------------------
    def leaf_hamiltonian(self, n_sites: int, terms):
        import torch

        arr, nt = make_terms(terms)
        ld = LeafDesc(n_sites, nt, arr)
        D = 1 << n_sites
        H = torch.empty((D, D), dtype=torch.float64, device=f"cuda:{self.device}")
        self._check(lib().rmc_leaf_hamiltonian(self.h, C.byref(ld), C.c_void_p(H.data_ptr())))
        return H

    def kron_apply(self, A: Module, B: Module, coefs, opA, opB, X, precision: int = FP64):
        import torch

        bd, keep = _bond(coefs, opA, opB)
        X = X.contiguous()
        Y = torch.empty_like(X)
        self._check(lib().rmc_kron_apply(self.h, A.h, B.h, C.byref(bd), int(precision),
                                         int(X.shape[0]), C.c_void_p(X.data_ptr()),
                                         C.c_void_p(Y.data_ptr())))
        return Y

    def kron_apply_noalloc(self, A: Module, B: Module, coefs, opA, opB, X, Y,
                           precision: int = FP64):
        """rmc_kron_apply_noalloc into the caller's Y (device tensor shaped like X):
        enqueued on the context's stream, nothing allocated, no synchronisation."""
        bd, keep = _bond(coefs, opA, opB)
        assert X.is_contiguous() and Y.is_contiguous() and X.shape == Y.shape
        self._check(lib().rmc_kron_apply_noalloc(self.h, A.h, B.h, C.byref(bd), int(precision),
                                                 int(X.shape[0]), C.c_void_p(X.data_ptr()),
                                                 C.c_void_p(Y.data_ptr())))
        return Y

    def sym_eig(self, A):
        import torch

        A = A.contiguous()
        b, m, _ = A.shape
        ev = torch.empty((b, m), dtype=torch.float64, device=A.device)
        V = torch.empty_like(A)
        self._check(lib().rmc_sym_eig(self.h, int(b), int(m), C.c_void_p(A.data_ptr()),
                                      C.c_void_p(ev.data_ptr()), C.c_void_p(V.data_ptr())))
        return ev, V


def job_chain(job):
    """(n_sites, leaf_sites, terms, k, q) for rmc_recurse from a workloads.ChainJob."""
    from .spin_models import chain_terms

    return (job.n_sites, job.leaf_sites, chain_terms(job), job.k, job.q)
