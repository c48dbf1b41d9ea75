"""ctypes binding of libbst.so (the C ABI declared in include/bst.h).

Argument marshalling only: every step of the compute path runs in the HIP
library.  torch supplies device memory and streams.  If the library is not
built, importing this module raises ImportError; there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os
import weakref
from typing import List, Sequence, Tuple

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
# BST_LIB may name another build of the same library (the host-sanitized
# build used by the test suite); by default the in-tree libbst.so.
LIB_PATH = os.environ.get("BST_LIB") or os.path.join(HERE, "libbst.so")

STATUS = {0: "OK", 1: "E_INVALID", 2: "E_DIRECTION", 3: "E_QNUM", 4: "E_DIM", 5: "E_LABEL",
          6: "E_NOBLOCK", 7: "E_STRUCTURE", 8: "E_DEVICE", 9: "E_NOTCONV"}
PREC = {"fp64": 0, "fp32": 1, "bf16x3": 2, "bf16x6": 3}
STATIC_WORKSPACE_BYTES = 64 << 20   # BST_STATIC_WORKSPACE_BYTES

# Every symbol include/bst.h declares.
EXPORTS = [
    "bst_tensor_create", "bst_tensor_destroy", "bst_tensor_info", "bst_tensor_leg",
    "bst_tensor_block", "bst_tensor_find_block", "bst_permute_plan", "bst_contract_plan",
    "bst_heff_plan", "bst_heff_batch_plan", "bst_plan_workspace", "bst_plan_info",
    "bst_plan_step_info", "bst_plan_set_precision", "bst_plan_use_graph", "bst_execute",
    "bst_plan_autotune", "bst_plan_tiles", "bst_plan_profile", "bst_plan_destroy",
    "bst_lanczos_workspace", "bst_lanczos_ground", "bst_last_error", "bst_version",
    "bst_plan_tile_count", "bst_plan_set_tile", "bst_plan_forget_workspace",
    "bst_tensor_create_sym", "bst_tensor_symmetry", "bst_tensor_leg_charges",
    "bst_network_order", "bst_plan_record_tiles", "bst_execute_static", "bst_calib_grid", "bst_calib_copy", "bst_calib_read", "bst_calib_mfma",
    "bst_svd_plan", "bst_svd_info", "bst_svd_sector", "bst_svd_execute", "bst_svd_truncate",
    "bst_svd_factors", "bst_svd_write", "bst_svd_sweeps", "bst_svd_forget_workspace", "bst_svd_destroy",
    "bst_permute_plan_c128", "bst_contract_plan_c128",
]


class BstError(RuntimeError):
    def __init__(self, status: int, msg: str):
        self.status = STATUS.get(status, str(status))
        super().__init__(f"{self.status}: {msg}")


class PlanStats(C.Structure):
    _fields_ = [("flops", C.c_double), ("gemm_flops", C.c_double), ("bytes", C.c_double),
                ("gemm_problems", C.c_int64), ("gemm_tiles", C.c_int64), ("launches", C.c_int64),
                ("nsteps", C.c_int32)]


class StepInfo(C.Structure):
    _fields_ = [("name", C.c_char * 32), ("flops", C.c_double), ("bytes_fp64", C.c_double),
                ("bytes_fp32", C.c_double), ("items", C.c_int64)]


class LanczosInfo(C.Structure):
    _fields_ = [("flags", C.c_int32), ("steps", C.c_int32), ("theta", C.c_double),
                ("beta_min", C.c_double), ("residual", C.c_double), ("alpha", C.c_double * 128),
                ("beta", C.c_double * 128), ("kernel_ms", C.c_double * 8),
                ("kernel_calls", C.c_int32 * 8)]


# Kernel classes of the timing record.  Default schedule: gs_dots is the
# u_j.z dot, gs_update the single pass over the basis, gs_third unused;
# three-pass schedule: V^T w, project + V^T w, project + norm.
LANCZOS_KERNEL_CLASSES = ["gemm_L_psi", "mpo_apply", "gemm_T3_R", "prep", "gs_dots",
                          "gs_update", "gs_third", "vector_other"]


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run paper_2401_01921_amd.build")
    lib = C.CDLL(LIB_PATH)
    vp, i32, i64, sz = C.c_void_p, C.c_int32, C.c_int64, C.c_size_t
    P = C.POINTER
    sig = {
        "bst_tensor_create": [i32, P(i32), P(i32), P(i32), P(i64), P(C.c_char_p), P(vp)],
        "bst_tensor_create_sym": [i32, P(i32), P(i32), i32, P(i32), P(i32), P(i64), P(C.c_char_p),
                                  P(vp)],
        "bst_tensor_symmetry": [vp, P(i32), P(i32), i32],
        "bst_tensor_leg_charges": [vp, i32, P(i32)],
        "bst_network_order": [i32, P(i32), P(i32), i32, P(i64), P(i32), P(C.c_double)],
        "bst_tensor_destroy": [vp],
        "bst_tensor_info": [vp, P(i32), P(i64), P(i64)],
        "bst_tensor_leg": [vp, i32, P(i32), P(i32), P(i32), P(i64), C.c_char_p, sz],
        "bst_tensor_block": [vp, i64, P(i32), P(i64), P(i64)],
        "bst_tensor_find_block": [vp, P(i32), P(i64)],
        "bst_permute_plan": [vp, P(C.c_char_p), P(vp), P(vp)],
        "bst_contract_plan": [vp, vp, C.c_int, P(vp), P(vp)],
        "bst_heff_plan": [vp, vp, vp, vp, vp, C.c_int, P(vp)],
        "bst_heff_batch_plan": [i32, P(vp), P(vp)],
        "bst_plan_workspace": [vp, P(sz)],
        "bst_plan_info": [vp, P(PlanStats)],
        "bst_plan_step_info": [vp, i32, P(StepInfo)],
        "bst_plan_set_precision": [vp, C.c_int],
        "bst_plan_use_graph": [vp, i32],
        "bst_execute": [vp, P(vp), P(vp), vp, vp],
        "bst_execute_static": [vp, P(vp), P(vp), vp],
        "bst_plan_autotune": [vp, P(vp), P(vp), vp, vp, i32],
        "bst_plan_tiles": [vp, C.c_char_p, sz],
        "bst_plan_tile_count": [vp, C.c_int, P(i32)],
        "bst_plan_set_tile": [vp, C.c_int, i32],
        "bst_plan_record_tiles": [vp],
        "bst_plan_profile": [vp, P(vp), P(vp), vp, vp, i32, P(C.c_double), i32, P(i32)],
        "bst_plan_destroy": [vp],
        "bst_plan_forget_workspace": [vp],
        "bst_lanczos_workspace": [vp, i32, P(sz)],
        "bst_lanczos_ground": [vp, P(vp), vp, i32, C.c_int, i32, vp, P(C.c_double),
                               P(LanczosInfo), vp, vp],
    }
    sig.update({
        "bst_calib_copy": [vp, vp, sz, vp],
        "bst_calib_read": [vp, sz, vp, vp],
        "bst_calib_mfma": [C.c_int, i64, vp, P(C.c_double), vp],
    })
    sig.update({
        "bst_svd_plan": [vp, i32, P(vp)],
        "bst_svd_info": [vp, P(i32), P(i64), P(sz)],
        "bst_svd_sector": [vp, i32, P(i32), P(i64), P(i64)],
        "bst_svd_execute": [vp, vp, vp, vp],
        "bst_svd_truncate": [vp, i64, C.c_double, P(i64), vp, vp, P(i64), P(C.c_double)],
        "bst_svd_factors": [vp, P(i64), C.c_char_p, P(vp), P(vp)],
        "bst_svd_write": [vp, P(i64), i32, vp, vp, vp, vp, vp],
        "bst_svd_sweeps": [vp, vp, vp, P(i32)],
        "bst_svd_forget_workspace": [vp],
        "bst_svd_destroy": [vp],
        "bst_permute_plan_c128": [vp, P(C.c_char_p), P(vp), P(vp)],
        "bst_contract_plan_c128": [vp, vp, C.c_int, P(vp), P(vp)],
    })
    for name, args in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = C.c_int
    lib.bst_last_error.restype = C.c_char_p
    lib.bst_last_error.argtypes = []
    lib.bst_calib_grid.restype = C.c_int32
    lib.bst_calib_grid.argtypes = []
    lib.bst_version.restype = C.c_char_p
    lib.bst_version.argtypes = []
    return lib


_lib = _load()


def lib():
    return _lib


def _check(status: int):
    if status != 0:
        raise BstError(status, _lib.bst_last_error().decode())


def version() -> str:
    return _lib.bst_version().decode()


def _prec(p) -> int:
    return PREC[p] if isinstance(p, str) else int(p)


# --------------------------------------------------------------------------
class Tensor:
    """Descriptor of a block-sparse tensor: labels and legs ``(dir, [(q, g), ...])``.

    ``sym`` lists the symmetries (0 for U(1), n for Z_n); the default is one
    U(1).  With several symmetries each charge ``q`` is a tuple, one entry
    per symmetry."""

    def __init__(self, labels: Sequence[str], legs, _handle=None, sym: Sequence[int] | None = None):
        if _handle is not None:
            self._h = _handle
        else:
            rank = len(legs)
            if len(labels) != rank:
                raise BstError(1, "one label per leg")
            dirs = (C.c_int32 * max(rank, 1))(*[int(d) for d, _ in legs])
            nsec = (C.c_int32 * max(rank, 1))(*[len(s) for _, s in legs])
            gs = [int(g) for _, s in legs for _, g in s]
            dm = (C.c_int64 * max(len(gs), 1))(*gs)
            labs = (C.c_char_p * max(rank, 1))(*[l.encode() for l in labels])
            h = C.c_void_p()
            if sym is None:
                qs = [int(q) for _, s in legs for q, _ in s]
                qn = (C.c_int32 * max(len(qs), 1))(*qs)
                _check(_lib.bst_tensor_create(rank, dirs, nsec, qn, dm, labs, C.byref(h)))
            else:
                ns = len(sym)
                qs = [int(c) for _, s in legs for q, _ in s
                      for c in (q if isinstance(q, (tuple, list)) else (q,))]
                if len(qs) != ns * len(gs):
                    raise BstError(1, "one charge per symmetry and sector")
                qn = (C.c_int32 * max(len(qs), 1))(*qs)
                sy = (C.c_int32 * ns)(*[int(m) for m in sym])
                _check(_lib.bst_tensor_create_sym(rank, dirs, nsec, ns, sy, qn, dm, labs, C.byref(h)))
            self._h = h
        r, nb, ne = C.c_int32(), C.c_int64(), C.c_int64()
        _check(_lib.bst_tensor_info(self._h, C.byref(r), C.byref(nb), C.byref(ne)))
        self.rank, self.nblocks, self.numel = r.value, nb.value, ne.value
        self._table = None

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and _lib is not None:
            _lib.bst_tensor_destroy(h)
            self._h = None

    @property
    def handle(self):
        return self._h

    def legs(self):
        out, labels = [], []
        for i in range(self.rank):
            d, ns = C.c_int32(), C.c_int32()
            _check(_lib.bst_tensor_leg(self._h, i, C.byref(d), C.byref(ns), None, None, None, 0))
            qn = (C.c_int32 * ns.value)()
            dm = (C.c_int64 * ns.value)()
            lab = C.create_string_buffer(256)
            _check(_lib.bst_tensor_leg(self._h, i, None, None, qn, dm, lab, 256))
            out.append((d.value, list(zip(list(qn), list(dm)))))
            labels.append(lab.value.decode())
        return labels, out

    @property
    def labels(self) -> List[str]:
        return self.legs()[0]

    def symmetry(self) -> List[int]:
        """Moduli of the symmetries (0 = U(1))."""
        n = C.c_int32()
        m = (C.c_int32 * 8)()
        _check(_lib.bst_tensor_symmetry(self._h, C.byref(n), m, 8))
        return list(m[:n.value])

    def leg_charges(self, leg: int) -> List[Tuple[int, ...]]:
        """Every sector's charges (one per symmetry) of a leg."""
        ns = len(self.symmetry())
        d, nsec = C.c_int32(), C.c_int32()
        _check(_lib.bst_tensor_leg(self._h, leg, C.byref(d), C.byref(nsec), None, None, None, 0))
        q = (C.c_int32 * max(nsec.value * ns, 1))()
        _check(_lib.bst_tensor_leg_charges(self._h, leg, q))
        return [tuple(q[k * ns:(k + 1) * ns]) for k in range(nsec.value)]

    def table(self) -> List[Tuple[Tuple[int, ...], Tuple[int, ...], int]]:
        """[(sector indices, shape, flat offset)] in canonical block order."""
        if self._table is None:
            r = max(self.rank, 1)
            qi = (C.c_int32 * r)()
            sh = (C.c_int64 * r)()
            off = C.c_int64()
            t = []
            for b in range(self.nblocks):
                _check(_lib.bst_tensor_block(self._h, b, qi, sh, C.byref(off)))
                t.append((tuple(qi[:self.rank]), tuple(sh[:self.rank]), off.value))
            self._table = t
        return self._table

    def find_block(self, qn_idx: Sequence[int]) -> int:
        qi = (C.c_int32 * max(self.rank, 1))(*qn_idx)
        b = C.c_int64()
        _check(_lib.bst_tensor_find_block(self._h, qi, C.byref(b)))
        return b.value

    # host-side marshalling between a dense array and the flat block layout
    def _sector_starts(self):
        _, legs = self.legs()
        return [np.concatenate([[0], np.cumsum([g for _, g in s])[:-1]]).astype(int) for _, s in legs]

    def from_dense(self, dense: np.ndarray) -> np.ndarray:
        starts = self._sector_starts()
        flat = np.zeros(self.numel)
        for qi, sh, off in self.table():
            sl = tuple(slice(starts[i][k], starts[i][k] + sh[i]) for i, k in enumerate(qi))
            flat[off:off + int(np.prod(sh))] = np.asarray(dense[sl], dtype=np.float64).ravel()
        return flat

    def to_dense(self, flat: np.ndarray) -> np.ndarray:
        _, legs = self.legs()
        dense = np.zeros([sum(g for _, g in s) for _, s in legs])
        starts = self._sector_starts()
        for qi, sh, off in self.table():
            sl = tuple(slice(starts[i][k], starts[i][k] + sh[i]) for i, k in enumerate(qi))
            dense[sl] = np.asarray(flat[off:off + int(np.prod(sh))]).reshape(sh)
        return dense


# --------------------------------------------------------------------------
def _ptr(t) -> int:
    import torch
    if not isinstance(t, torch.Tensor):
        raise TypeError("device buffers are torch tensors")
    if t.numel() == 0:
        return 0
    if not t.is_cuda:
        raise ValueError("device buffers must live on the GPU")
    if not t.is_contiguous():
        raise ValueError("device buffers must be contiguous")
    return t.data_ptr()


def _stream(stream) -> C.c_void_p:
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return C.c_void_p(stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream))


def workspace(nbytes: int, device="cuda"):
    """A 256-byte aligned device byte buffer of at least nbytes."""
    import torch
    buf = torch.empty(int(nbytes) + 256, dtype=torch.uint8, device=device)
    shift = (-buf.data_ptr()) % 256
    return buf[shift:shift + int(nbytes)]


class Plan:
    def __init__(self, handle, n_in: int, n_out: int, in_numel=None, out_numel=None):
        self._h = handle
        self.n_in, self.n_out = n_in, n_out
        self.in_numel, self.out_numel = in_numel, out_numel
        b = C.c_size_t()
        _check(_lib.bst_plan_workspace(self._h, C.byref(b)))
        self.workspace_bytes = b.value

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and _lib is not None:
            _lib.bst_plan_destroy(h)
            self._h = None

    @property
    def handle(self):
        return self._h

    def stats(self) -> PlanStats:
        s = PlanStats()
        _check(_lib.bst_plan_info(self._h, C.byref(s)))
        return s

    def steps(self):
        out = []
        for k in range(self.stats().nsteps):
            si = StepInfo()
            _check(_lib.bst_plan_step_info(self._h, k, C.byref(si)))
            out.append(dict(name=si.name.decode(), flops=si.flops, bytes_fp64=si.bytes_fp64,
                            bytes_fp32=si.bytes_fp32, items=si.items))
        return out

    def set_precision(self, prec):
        _check(_lib.bst_plan_set_precision(self._h, _prec(prec)))

    def use_graph(self, on: bool = True):
        _check(_lib.bst_plan_use_graph(self._h, 1 if on else 0))

    def tile_count(self, prec) -> int:
        n = C.c_int32()
        _check(_lib.bst_plan_tile_count(self._h, _prec(prec), C.byref(n)))
        return n.value

    def set_tile(self, prec, tile: int):
        _check(_lib.bst_plan_set_tile(self._h, _prec(prec), tile))

    def record_tiles(self):
        """Write the chosen tile shapes into the BST_TUNE_CACHE file."""
        _check(_lib.bst_plan_record_tiles(self._h))

    def tiles(self) -> str:
        buf = C.create_string_buffer(4096)
        _check(_lib.bst_plan_tiles(self._h, buf, 4096))
        return buf.value.decode()

    def _arrays(self, ins, outs):
        if len(ins) != self.n_in or len(outs) != self.n_out:
            raise BstError(1, f"plan takes {self.n_in} inputs and {self.n_out} outputs")
        import torch
        for k, t in enumerate(list(ins) + list(outs)):
            if t.dtype != torch.float64:
                raise BstError(1, f"buffer {k} must be float64")
        if self.in_numel is not None:
            for k, (t, n) in enumerate(zip(ins, self.in_numel)):
                if n is not None and t.numel() != n:
                    raise BstError(1, f"input {k} has {t.numel()} elements, expected {n}")
        if self.out_numel is not None:
            for k, (t, n) in enumerate(zip(outs, self.out_numel)):
                if n is not None and t.numel() != n:
                    raise BstError(1, f"output {k} has {t.numel()} elements, expected {n}")
        a = (C.c_void_p * max(len(ins), 1))(*[_ptr(t) for t in ins])
        b = (C.c_void_p * max(len(outs), 1))(*[_ptr(t) for t in outs])
        return a, b

    def _check_ws(self, ws, need=None):
        need = self.workspace_bytes if need is None else need
        if ws.numel() * ws.element_size() < need:
            raise BstError(1, f"workspace has {ws.numel() * ws.element_size()} bytes, plan needs {need}")
        # The library keeps the plan's tables in the workspace between calls
        # and re-uploads them only when told to: do so whenever this is not
        # the workspace object of the previous call, or it was modified since.
        ref = getattr(self, "_ws_ref", None)
        if ref is None or ref() is not ws or getattr(self, "_ws_version", None) != ws._version:
            _check(_lib.bst_plan_forget_workspace(self._h))
            self._ws_ref = weakref.ref(ws)
            self._ws_version = ws._version

    def execute(self, ins, outs, ws, stream=None):
        self._check_ws(ws)
        a, b = self._arrays(ins, outs)
        _check(_lib.bst_execute(self._h, a, b, C.c_void_p(_ptr(ws)), _stream(stream)))

    def execute_static(self, ins, outs, stream=None):
        """execute() with the library's fixed per-device workspace
        (STATIC_WORKSPACE_BYTES): allocates nothing; calls overlapping on
        one device race."""
        a, b = self._arrays(ins, outs)
        _check(_lib.bst_execute_static(self._h, a, b, _stream(stream)))

    def autotune(self, ins, outs, ws, reps: int = 5, stream=None):
        self._check_ws(ws)
        a, b = self._arrays(ins, outs)
        _check(_lib.bst_plan_autotune(self._h, a, b, C.c_void_p(_ptr(ws)), _stream(stream), reps))

    def profile(self, ins, outs, ws, reps: int = 10, stream=None):
        self._check_ws(ws)
        a, b = self._arrays(ins, outs)
        cap = 64
        ms = (C.c_double * cap)()
        n = C.c_int32()
        _check(_lib.bst_plan_profile(self._h, a, b, C.c_void_p(_ptr(ws)), _stream(stream), reps,
                                     ms, cap, C.byref(n)))
        st = self.steps()
        return [(st[k]["name"], ms[k]) for k in range(n.value)]


def permute_plan(T: Tensor, order: Sequence[str], dtype: str = "f64"):
    """dtype "c128": complex data, two float64 per element (buffers of
    2 * numel doubles, e.g. torch.view_as_real(x).reshape(-1))."""
    labs = (C.c_char_p * max(len(order), 1))(*[l.encode() for l in order])
    h, p = C.c_void_p(), C.c_void_p()
    f = _lib.bst_permute_plan_c128 if dtype == "c128" else _lib.bst_permute_plan
    _check(f(T.handle, labs, C.byref(h), C.byref(p)))
    out = Tensor(None, None, _handle=h)
    w = 2 if dtype == "c128" else 1
    return out, Plan(p, 1, 1, [w * T.numel], [w * out.numel])


def contract_plan(A: Tensor, B: Tensor, prec="fp64", dtype: str = "f64"):
    h, p = C.c_void_p(), C.c_void_p()
    f = _lib.bst_contract_plan_c128 if dtype == "c128" else _lib.bst_contract_plan
    _check(f(A.handle, B.handle, _prec(prec), C.byref(h), C.byref(p)))
    out = Tensor(None, None, _handle=h)
    w = 2 if dtype == "c128" else 1
    return out, Plan(p, 2, 1, [w * A.numel, w * B.numel], [w * out.numel])


def heff_plan(L: Tensor, W1: Tensor, W2: Tensor, R: Tensor, psi: Tensor, prec="fp64") -> Plan:
    p = C.c_void_p()
    _check(_lib.bst_heff_plan(L.handle, W1.handle, W2.handle, R.handle, psi.handle, _prec(prec),
                              C.byref(p)))
    plan = Plan(p, 5, 1, [L.numel, W1.numel, W2.numel, R.numel, psi.numel], [psi.numel])
    plan.psi_numel = psi.numel
    return plan


def heff_batch_plan(plans: Sequence[Plan]) -> Plan:
    arr = (C.c_void_p * len(plans))(*[p.handle.value for p in plans])
    b = C.c_void_p()
    _check(_lib.bst_heff_batch_plan(len(plans), arr, C.byref(b)))
    ins, outs = [], []
    for p in plans:
        ins += p.in_numel
        outs += p.out_numel
    return Plan(b, 5 * len(plans), len(plans), ins, outs)


def lanczos_workspace(plan: Plan, nsteps: int) -> int:
    b = C.c_size_t()
    _check(_lib.bst_lanczos_workspace(plan.handle, nsteps, C.byref(b)))
    return b.value


def lanczos_ground(plan: Plan, ops, psi0, nsteps: int, prec="fp64", refine: bool = True,
                   ws=None, psi_out=None, stream=None, timing: bool = False,
                   three_pass: bool = False, f32_basis: bool = False):
    """ops = [L, W1, W2, R] device tensors; psi0 device tensor.  Returns a dict
    with energy, theta, steps, residual, beta_min, alpha, beta and psi.
    three_pass selects the textbook reorthogonalisation schedule (three passes
    over the basis per step) instead of the default single pass; f32_basis
    stores the Krylov rows as float32 with the bf16x3 / bf16x6 forms (float64
    rows by default)."""
    import torch
    if ws is None:
        ws = workspace(lanczos_workspace(plan, nsteps), psi0.device)
    if psi_out is None:
        psi_out = torch.empty_like(psi0)
    if psi0.numel() != plan.psi_numel or psi_out.numel() != plan.psi_numel:
        raise BstError(1, "psi0 / psi_out have the wrong size")
    plan._check_ws(ws, lanczos_workspace(plan, nsteps))
    for t, n in zip(ops, plan.in_numel[:4]):
        if t.numel() != n or t.dtype != torch.float64:
            raise BstError(1, "operator buffer has the wrong size or dtype")
    if psi0.dtype != torch.float64 or psi_out.dtype != torch.float64:
        raise BstError(1, "psi buffers must be float64")
    a = (C.c_void_p * 4)(*[_ptr(t) for t in ops])
    e = C.c_double()
    info = LanczosInfo()
    info.flags = (1 if timing else 0) | (2 if three_pass else 0) | (4 if f32_basis else 0)
    _check(_lib.bst_lanczos_ground(plan.handle, a, C.c_void_p(_ptr(psi0)), nsteps, _prec(prec),
                                   1 if refine else 0, C.c_void_p(_ptr(psi_out)), C.byref(e),
                                   C.byref(info), C.c_void_p(_ptr(ws)), _stream(stream)))
    m = info.steps
    out = dict(energy=e.value, theta=info.theta, steps=m, residual=info.residual,
               beta_min=info.beta_min, alpha=np.array(info.alpha[:m]), beta=np.array(info.beta[:m]),
               psi=psi_out, z32=bool(info.flags & 16))
    if timing:
        out["kernel_ms"] = {n: info.kernel_ms[i] for i, n in enumerate(LANCZOS_KERNEL_CLASSES)}
        out["kernel_calls"] = {n: info.kernel_calls[i] for i, n in enumerate(LANCZOS_KERNEL_CLASSES)}
    return out


# --------------------------------------------------------------------------
# calibration kernels (the device's practical streaming and MFMA rates)
def calib_grid() -> int:
    return int(_lib.bst_calib_grid())


def calib_copy(src, dst, stream=None):
    """Streaming copy of src into dst (device tensors of equal byte size)."""
    nb = src.numel() * src.element_size()
    if dst.numel() * dst.element_size() != nb:
        raise BstError(1, "copy buffers differ in size")
    _check(_lib.bst_calib_copy(C.c_void_p(_ptr(src)), C.c_void_p(_ptr(dst)), nb, _stream(stream)))


def calib_read(src, partial, stream=None):
    """Streaming read of src; partial (float64, calib_grid() elements) gets
    one sum per workgroup."""
    import torch
    if partial.dtype != torch.float64 or partial.numel() < calib_grid():
        raise BstError(1, "partial needs calib_grid() float64 elements")
    _check(_lib.bst_calib_read(C.c_void_p(_ptr(src)), src.numel() * src.element_size(),
                               C.c_void_p(_ptr(partial)), _stream(stream)))


def calib_mfma(prec, iters: int, out, stream=None) -> float:
    """Back-to-back MFMA loop in form prec ("fp64" or "bf16x3" for the
    bfloat16 instruction); out holds 256 * calib_grid() float64.  Returns the
    flops of the launch."""
    import torch
    if out.dtype != torch.float64 or out.numel() < 256 * calib_grid():
        raise BstError(1, "out needs 256 * calib_grid() float64 elements")
    f = C.c_double()
    _check(_lib.bst_calib_mfma(_prec(prec), int(iters), C.c_void_p(_ptr(out)), C.byref(f),
                               _stream(stream)))
    return f.value


# --------------------------------------------------------------------------
class Svd:
    """Plan of the SVD of one tensor structure (bst_svd_*): execute, then
    truncate, then factors / write.  Argument marshalling only."""

    def __init__(self, T: Tensor, rowrank: int):
        h = C.c_void_p()
        _check(_lib.bst_svd_plan(T.handle, int(rowrank), C.byref(h)))
        self._h = h
        ns, nv, ws = C.c_int32(), C.c_int64(), C.c_size_t()
        _check(_lib.bst_svd_info(self._h, C.byref(ns), C.byref(nv), C.byref(ws)))
        self.nsectors, self.nvalues, self.workspace_bytes = ns.value, nv.value, ws.value
        self.nsym = len(T.symmetry())

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and _lib is not None:
            _lib.bst_svd_destroy(h)
            self._h = None

    def sector(self, k: int):
        """(charge, rows, cols) of sector k of the new bond."""
        q = (C.c_int32 * max(self.nsym, 1))()
        r, c = C.c_int64(), C.c_int64()
        _check(_lib.bst_svd_sector(self._h, int(k), q, C.byref(r), C.byref(c)))
        ch = tuple(q[:self.nsym])
        return (ch if self.nsym > 1 else ch[0]), r.value, c.value

    def execute(self, M, ws, stream=None):
        _check(_lib.bst_svd_execute(self._h, C.c_void_p(_ptr(M)), C.c_void_p(_ptr(ws)), _stream(stream)))

    def truncate(self, keepdim: int, err: float = 0.0, min_blockdim=None, ws=None, stream=None):
        """Kept count per sector and the largest value not kept (blocks)."""
        kept = (C.c_int64 * max(self.nsectors, 1))()
        se = C.c_double()
        mb = None
        if min_blockdim is not None:
            if len(min_blockdim) != self.nsectors:
                raise BstError(1, "one min_blockdim entry per sector")
            mb = (C.c_int64 * max(self.nsectors, 1))(*[int(x) for x in min_blockdim])
        _check(_lib.bst_svd_truncate(self._h, int(keepdim), float(err), mb, C.c_void_p(_ptr(ws)),
                                     _stream(stream), kept, C.byref(se)))
        return list(kept[:self.nsectors]), se.value

    def factors(self, kept, bond: str):
        """(U, V^dagger) descriptors for the kept counts."""
        k = (C.c_int64 * max(self.nsectors, 1))(*[int(x) for x in kept])
        u, v = C.c_void_p(), C.c_void_p()
        _check(_lib.bst_svd_factors(self._h, k, bond.encode(), C.byref(u), C.byref(v)))
        return Tensor(None, None, _handle=u), Tensor(None, None, _handle=v)

    def write(self, kept, absorb: int, U, S, Vd, ws, stream=None):
        k = (C.c_int64 * max(self.nsectors, 1))(*[int(x) for x in kept])
        _check(_lib.bst_svd_write(self._h, k, int(absorb), C.c_void_p(_ptr(U)), C.c_void_p(_ptr(S)),
                                  C.c_void_p(_ptr(Vd)), C.c_void_p(_ptr(ws)), _stream(stream)))

    def sweeps(self, ws, stream=None):
        """Jacobi sweeps each sector used in the last execute on ws."""
        out = (C.c_int32 * max(self.nsectors, 1))()
        _check(_lib.bst_svd_sweeps(self._h, C.c_void_p(_ptr(ws)), _stream(stream), out))
        return [int(x) for x in out[:self.nsectors]]

    def forget_workspace(self):
        _check(_lib.bst_svd_forget_workspace(self._h))


ABSORB = {None: 0, "u": 1, "v": 2}


def svd_truncate(T: Tensor, M, rowrank: int, keepdim: int, err: float = 0.0, min_blockdim=None,
                 bond: str = "_m", absorb=None, device="cuda"):
    """Svd_truncate of the device tensor M (structure T): returns
    (U descriptor, U data, S data, V^dagger descriptor, V^dagger data, s_err,
    kept counts), data as float64 device tensors."""
    import torch
    plan = Svd(T, rowrank)
    ws = workspace(plan.workspace_bytes, device)
    plan.execute(M, ws)
    kept, s_err = plan.truncate(keepdim, err, min_blockdim, ws)
    Ut, Vt = plan.factors(kept, bond)
    U = torch.empty(Ut.numel, dtype=torch.float64, device=device)
    Vd = torch.empty(Vt.numel, dtype=torch.float64, device=device)
    S = torch.empty(max(sum(kept), 1), dtype=torch.float64, device=device)[:sum(kept)]
    plan.write(kept, ABSORB[absorb], U, S, Vd, ws)
    return Ut, U, S, Vt, Vd, s_err, kept
