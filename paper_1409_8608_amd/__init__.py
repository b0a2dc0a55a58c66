"""Python binding of libtc (MI355X tensor contractions).

Argument marshalling only: every step of a contraction runs in libtc.so (host
planning in C++, all arithmetic in HIP kernels).  PyTorch supplies device
memory and streams.  The functions ``tc_plan``, ``tc_contract``, ... mirror the
C ABI in ``include/tc.h`` one to one; ``Plan`` and ``Batch`` wrap them.

Importing this package loads libtc.so and raises if it is missing: there is no
fallback path.  Build it with ``python paper_1409_8608_amd/build.py``.
"""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libtc.so")

TC_F64, TC_F32, TC_C128, TC_C64 = 0, 1, 2, 3
DTYPES = dict(f64=TC_F64, f32=TC_F32, c128=TC_C128, c64=TC_C64)
TC_NATIVE, TC_BF16X3, TC_FP8X3 = 0, 1, 2
TC_VARIANT_FUSED, TC_VARIANT_PREDICTED = -2, -1
KERNELS = ("dot", "axpy", "gemv", "ger", "gemm", "fused")
STATUS = ("TC_OK", "TC_E_SPEC", "TC_E_EXTENT", "TC_E_STRIDE", "TC_E_DTYPE", "TC_E_ALIAS", "TC_E_NULL",
          "TC_E_VARIANT", "TC_E_HIP", "TC_E_NOMEM", "TC_E_UNSUPPORTED", "TC_E_CAPACITY")
TC_MAX_SETUP = 16
EXPORTS = ("tc_plan", "tc_plan_destroy", "tc_variant_count", "tc_variant_get", "tc_set_variant",
           "tc_plan_prepare", "tc_plan_workspace", "tc_contract", "tc_contract_complex", "tc_access_distance", "tc_bench_classes",
           "tc_predict", "tc_batch_create", "tc_batch_tune", "tc_batch_contract", "tc_batch_destroy",
           "tc_batch_info", "tc_split_terms", "tc_status_str", "tc_last_error", "tc_set_root_gap",
           "tc_chain_root_gaps", "tc_contract_noalloc", "tc_batch_score", "tc_batch_choice",
           "tc_batch_set_choice", "tc_set_split_products")


class TcError(RuntimeError):
    def __init__(self, status: int, detail: str):
        self.status = status
        self.name = STATUS[status] if 0 <= status < len(STATUS) else str(status)
        super().__init__(f"{self.name}: {detail}")


class tc_variant_info(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 40), ("number", ctypes.c_int), ("kernel", ctypes.c_int),
                ("kept", ctypes.c_char * 8), ("loops", ctypes.c_char * 16), ("n_copies", ctypes.c_int),
                ("copy_tensor", ctypes.c_char * 4), ("copy_level", ctypes.c_int * 4),
                ("n_hoisted", ctypes.c_int), ("launches", ctypes.c_int64), ("invocations", ctypes.c_int64),
                ("runs_on_gpu", ctypes.c_int)]


class tc_setup_item(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int), ("tensor", ctypes.c_int), ("size", ctypes.c_int64)]


class tc_bench_class(ctypes.Structure):
    _fields_ = [("label", ctypes.c_char * 16), ("weight", ctypes.c_double), ("n_items", ctypes.c_int),
                ("items", tc_setup_item * TC_MAX_SETUP)]


class tc_tune_score(ctypes.Structure):
    _fields_ = [("n_sampled", ctypes.c_int), ("candidates_mean", ctypes.c_double),
                ("within5_seed", ctypes.c_double), ("argmin_seed", ctypes.c_double), ("regret_seed", ctypes.c_double),
                ("within5_tuned", ctypes.c_double), ("argmin_tuned", ctypes.c_double),
                ("regret_tuned", ctypes.c_double), ("within5_default", ctypes.c_double),
                ("argmin_default", ctypes.c_double), ("regret_default", ctypes.c_double),
                ("member_best_share", ctypes.c_double), ("within5_topk", ctypes.c_double),
                ("argmin_topk", ctypes.c_double), ("regret_topk", ctypes.c_double)]


class tc_prediction(ctypes.Structure):
    _fields_ = [("variant", ctypes.c_int), ("predicted_s", ctypes.c_double), ("stage_s", ctypes.c_double * 5),
                ("bench_s", ctypes.c_double), ("n_bench", ctypes.c_int)]


def _load():
    # One HIP runtime per process: PyTorch ships its own libamdhip64 with the
    # same soname, and device pointers and streams from torch are only valid in
    # that runtime.  Importing torch first makes libtc bind to it.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"libtc.so not found at {LIB_PATH}: build it with "
                          "`python paper_1409_8608_amd/build.py` (there is no fallback path)")
    lib = ctypes.CDLL(LIB_PATH)
    P, I64P, D = ctypes.c_void_p, ctypes.POINTER(ctypes.c_int64), ctypes.c_double
    sig = {
        "tc_plan": [ctypes.POINTER(P), ctypes.c_char_p, ctypes.c_char_p, I64P, ctypes.c_int, I64P, I64P, I64P,
                    ctypes.c_int, ctypes.c_int],
        "tc_plan_destroy": [P],
        "tc_variant_count": [P, ctypes.POINTER(ctypes.c_int)],
        "tc_variant_get": [P, ctypes.c_int, ctypes.POINTER(tc_variant_info)],
        "tc_set_variant": [P, ctypes.c_int],
        "tc_plan_prepare": [P],
        "tc_plan_workspace": [P, I64P],
        "tc_contract": [P, P, P, P, D, D, P],
        "tc_contract_complex": [P, P, P, P, D, D, D, D, P],
        "tc_contract_noalloc": [P, P, P, P, D, D, P],
        "tc_access_distance": [P, ctypes.c_int, ctypes.c_int, I64P],
        "tc_bench_classes": [P, ctypes.c_int, ctypes.c_int, D, ctypes.c_int, ctypes.POINTER(tc_bench_class),
                             ctypes.c_int, ctypes.POINTER(ctypes.c_int)],
        "tc_predict": [P, ctypes.POINTER(tc_prediction), ctypes.c_int, ctypes.POINTER(ctypes.c_int)],
        "tc_batch_create": [ctypes.POINTER(P), ctypes.POINTER(P), ctypes.c_int],
        "tc_batch_tune": [P, ctypes.c_int],
        "tc_batch_contract": [P, ctypes.POINTER(P), ctypes.POINTER(P), ctypes.POINTER(P),
                              ctypes.POINTER(D), ctypes.POINTER(D), P],
        "tc_batch_destroy": [P],
        "tc_batch_score": [P, ctypes.c_int, ctypes.c_uint64, ctypes.POINTER(tc_tune_score)],
        "tc_batch_choice": [P, ctypes.c_int, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int),
                            ctypes.POINTER(ctypes.c_int)],
        "tc_batch_set_choice": [P, ctypes.c_int, ctypes.c_int, ctypes.c_int],
        "tc_batch_info": [P, ctypes.POINTER(ctypes.c_int), I64P, ctypes.POINTER(ctypes.c_int),
                          ctypes.POINTER(ctypes.c_double)],
        "tc_split_terms": [P, ctypes.c_int, P, ctypes.POINTER(ctypes.c_int32), I64P, I64P],
        "tc_set_split_products": [P, ctypes.c_int],
        "tc_set_root_gap": [P, I64P],
        "tc_chain_root_gaps": [ctypes.POINTER(P), ctypes.POINTER(ctypes.c_int), ctypes.c_int],
    }
    for name, args in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = ctypes.c_int
    lib.tc_status_str.argtypes = [ctypes.c_int]
    lib.tc_status_str.restype = ctypes.c_char_p
    lib.tc_last_error.argtypes = []
    lib.tc_last_error.restype = ctypes.c_char_p
    return lib


lib = _load()


def _check(status: int):
    if status != 0:
        raise TcError(status, lib.tc_last_error().decode(errors="replace"))


def _i64(seq):
    if seq is None:
        return None
    seq = [int(x) for x in seq]
    return (ctypes.c_int64 * max(1, len(seq)))(*seq)


# ---- one-to-one wrappers of the C ABI --------------------------------------------
def tc_plan(spec: str, extents: dict, strides_A=None, strides_B=None, strides_C=None,
            dtype: int = TC_F64, compute: int = TC_NATIVE) -> int:
    chars = "".join(sorted(extents))
    h = ctypes.c_void_p()
    _check(lib.tc_plan(ctypes.byref(h), spec.encode(), chars.encode(), _i64([extents[c] for c in chars]),
                       len(chars), _i64(strides_A), _i64(strides_B), _i64(strides_C), int(dtype), int(compute)))
    return h.value


def tc_plan_destroy(h):
    _check(lib.tc_plan_destroy(h))


def tc_variant_count(h) -> int:
    n = ctypes.c_int()
    _check(lib.tc_variant_count(h, ctypes.byref(n)))
    return n.value


def tc_variant_get(h, variant: int) -> dict:
    info = tc_variant_info()
    _check(lib.tc_variant_get(h, int(variant), ctypes.byref(info)))
    return dict(index=variant, name=info.name.decode(), number=info.number, kernel=KERNELS[info.kernel],
                kept=info.kept.decode(), loops=info.loops.decode(),
                copies=[(info.copy_tensor[c].decode() if isinstance(info.copy_tensor[c], bytes)
                         else chr(info.copy_tensor[c]), info.copy_level[c]) for c in range(info.n_copies)],
                n_hoisted=info.n_hoisted, launches=info.launches, invocations=info.invocations,
                runs_on_gpu=bool(info.runs_on_gpu))


def tc_set_variant(h, variant: int):
    _check(lib.tc_set_variant(h, int(variant)))


def tc_plan_prepare(h):
    _check(lib.tc_plan_prepare(h))


def tc_plan_workspace(h) -> int:
    n = ctypes.c_int64()
    _check(lib.tc_plan_workspace(h, ctypes.byref(n)))
    return n.value


def tc_contract(h, A_ptr: int, B_ptr: int, C_ptr: int, alpha: float = 1.0, beta: float = 0.0, stream: int = 0):
    _check(lib.tc_contract(h, A_ptr or None, B_ptr or None, C_ptr or None, float(alpha), float(beta),
                           stream or None))


def tc_contract_noalloc(h, A_ptr: int, B_ptr: int, C_ptr: int, alpha: float = 1.0, beta: float = 0.0,
                        stream: int = 0):
    _check(lib.tc_contract_noalloc(h, A_ptr or None, B_ptr or None, C_ptr or None, float(alpha), float(beta),
                                   stream or None))


def tc_contract_complex(h, A_ptr: int, B_ptr: int, C_ptr: int, alpha: complex = 1.0, beta: complex = 0.0,
                        stream: int = 0):
    al, be = complex(alpha), complex(beta)
    _check(lib.tc_contract_complex(h, A_ptr or None, B_ptr or None, C_ptr or None, al.real, al.imag, be.real,
                                   be.imag, stream or None))


def tc_access_distance(h, variant: int, tensor: int) -> int:
    n = ctypes.c_int64()
    _check(lib.tc_access_distance(h, int(variant), int(tensor), ctypes.byref(n)))
    return n.value


def tc_bench_classes(h, variant: int, stage: int, cache_elems: float, line_elems: int) -> list:
    cap = 16
    arr = (tc_bench_class * cap)()
    n = ctypes.c_int()
    _check(lib.tc_bench_classes(h, int(variant), int(stage), float(cache_elems), int(line_elems), arr, cap,
                                ctypes.byref(n)))
    out = []
    for c in arr[:n.value]:
        items = []
        for it in c.items[:c.n_items]:
            items.append(("op", "ABC"[it.tensor], it.size) if it.kind == 0 else ("remote", None, it.size))
        out.append(dict(label=c.label.decode(), weight=c.weight, setup=items))
    return out


def tc_set_root_gap(h, gaps=None):
    """gaps: three element counts (A, B, C), or None for the paper's assumption."""
    _check(lib.tc_set_root_gap(h, _i64(gaps) if gaps is not None else None))


def tc_chain_root_gaps(handles, ids):
    """handles: plans of the chain in run order; ids: 3 tensor ids per plan."""
    n = len(handles)
    ids = [int(x) for x in ids]
    if len(ids) != 3 * n:
        raise ValueError("tc_chain_root_gaps: three tensor ids per plan")
    _check(lib.tc_chain_root_gaps((ctypes.c_void_p * max(1, n))(*handles), (ctypes.c_int * max(1, 3 * n))(*ids), n))


def tc_predict(h) -> list:
    n = ctypes.c_int()
    st = lib.tc_predict(h, None, 0, ctypes.byref(n))
    if st not in (0, 11):
        _check(st)
    arr = (tc_prediction * max(1, n.value))()
    _check(lib.tc_predict(h, arr, n.value, ctypes.byref(n)))
    return [dict(variant=p.variant, predicted_s=p.predicted_s, stage_s=list(p.stage_s), bench_s=p.bench_s,
                 n_bench=p.n_bench) for p in arr[:n.value]]


def tc_batch_create(plans) -> int:
    arr = (ctypes.c_void_p * len(plans))(*plans)
    h = ctypes.c_void_p()
    _check(lib.tc_batch_create(ctypes.byref(h), arr, len(plans)))
    return h.value


def tc_batch_tune(h, top_k: int = 3):
    _check(lib.tc_batch_tune(h, int(top_k)))


def tc_batch_contract(h, A_ptrs, B_ptrs, C_ptrs, alphas, betas, stream: int = 0):
    n = len(A_ptrs)
    if not (len(B_ptrs) == len(C_ptrs) == len(alphas) == len(betas) == n):
        raise ValueError("tc_batch_contract: A, B, C, alpha and beta need one entry per batch member")
    members = ctypes.c_int()
    _check(lib.tc_batch_info(h, ctypes.byref(members), None, None, None))
    if n != members.value:
        raise ValueError(f"tc_batch_contract: {n} entries for a batch of {members.value} members")
    P = ctypes.c_void_p * max(1, n)
    D = ctypes.c_double * max(1, n)
    nul = lambda v: [x or None for x in v]
    _check(lib.tc_batch_contract(h, P(*nul(A_ptrs)), P(*nul(B_ptrs)), P(*nul(C_ptrs)), D(*alphas), D(*betas),
                                 stream or None))


def tc_batch_score(h, sample: int = 256, seed: int = 51) -> dict:
    sc = tc_tune_score()
    _check(lib.tc_batch_score(h, int(sample), int(seed), ctypes.byref(sc)))
    return {name: getattr(sc, name) for name, _ in tc_tune_score._fields_}


def tc_batch_choice(h, member: int) -> dict:
    v, sh, nc = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
    _check(lib.tc_batch_choice(h, int(member), ctypes.byref(v), ctypes.byref(sh), ctypes.byref(nc)))
    return dict(variant=v.value, shape=sh.value, candidates=nc.value)


def tc_batch_set_choice(h, member: int, variant: int, shape: int):
    _check(lib.tc_batch_set_choice(h, int(member), int(variant), int(shape)))


def tc_batch_destroy(h):
    _check(lib.tc_batch_destroy(h))


def tc_batch_info(h) -> dict:
    n, g = ctypes.c_int(), ctypes.c_int()
    t = ctypes.c_int64()
    r = ctypes.c_double()
    _check(lib.tc_batch_info(h, ctypes.byref(n), ctypes.byref(t), ctypes.byref(g), ctypes.byref(r)))
    return dict(members=n.value, tiles=t.value, groups=g.value, tune_hit_rate=r.value)


class Batch:
    """Many contractions in one graph launch; ``plans`` must outlive it."""

    def __init__(self, plans):
        self.plans = list(plans)
        self.handle = tc_batch_create([p.handle for p in self.plans])

    def __del__(self):
        h = getattr(self, "handle", None)
        if h:
            try:
                lib.tc_batch_destroy(h)
            except Exception:
                pass
            self.handle = None

    class Bound:
        """Operands of every member, checked once against the plans, with the
        pointer and scalar arrays of the C call built ahead: replaying a bound
        set costs one library call and no Python work per member."""

        def __init__(self, batch, As, Bs, Cs, alphas, betas):
            n = len(batch.plans)
            alphas = [1.0] * n if alphas is None else [float(x) for x in alphas]
            betas = [0.0] * n if betas is None else [float(x) for x in betas]
            if not (len(As) == len(Bs) == len(Cs) == len(alphas) == len(betas) == n):
                raise ValueError(f"Batch.contract: {n} members need {n} entries of A, B, C, alpha and beta")
            for p, A, B, C in zip(batch.plans, As, Bs, Cs):
                p.check_tensors(A, B, C, device=False)
            for p, A, B, C in zip(batch.plans, As, Bs, Cs):
                p.check_tensors(A, B, C)
            self.tensors = (list(As), list(Bs), list(Cs))          # kept alive while bound
            ptr = lambda x: (x.data_ptr() or None) if x is not None else None   # None: not read (alpha = 0)
            P, D = ctypes.c_void_p * max(1, n), ctypes.c_double * max(1, n)
            self.args = (P(*[ptr(x) for x in As]), P(*[ptr(x) for x in Bs]), P(*[ptr(x) for x in Cs]),
                         D(*alphas), D(*betas))

    def bind(self, As, Bs, Cs, alphas=None, betas=None):
        """Check the operands once; ``run`` then replays them."""
        return Batch.Bound(self, As, Bs, Cs, alphas, betas)

    def run(self, bound, stream=None):
        import torch
        if stream is None:
            stream = torch.cuda.current_stream().cuda_stream
        _check(lib.tc_batch_contract(self.handle, *bound.args, stream or None))

    def contract(self, As, Bs, Cs, alphas=None, betas=None, stream=None):
        """Check every member's tensors (dtype, shape, strides, device) and run
        the batch; use ``bind`` and ``run`` to replay the same operands."""
        self.run(self.bind(As, Bs, Cs, alphas, betas), stream)

    def tune(self, top_k: int = 2):
        tc_batch_tune(self.handle, top_k)

    def score(self, sample: int = 256, seed: int = 51):
        return tc_batch_score(self.handle, sample, seed)

    def choice(self, member: int):
        return tc_batch_choice(self.handle, member)

    def set_choice(self, member: int, variant: int, shape: int):
        tc_batch_set_choice(self.handle, member, variant, shape)

    def info(self):
        return tc_batch_info(self.handle)


def tc_split_terms(h, side: int, fp8: bool = False):
    """(terms [3, rows, kp], exponents int32 [rows]) of the last split contraction:
    BF16 bit patterns (uint16), or E4M3 codes (uint8) with ``fp8`` for a
    TC_FP8X3 plan, term p stored scaled by 2^(4(p-1))."""
    import numpy as np
    rows, kp = ctypes.c_int64(), ctypes.c_int64()
    _check(lib.tc_split_terms(h, int(side), None, None, ctypes.byref(rows), ctypes.byref(kp)))
    terms = np.zeros((3, rows.value, kp.value), dtype=np.uint8 if fp8 else np.uint16)
    exps = np.zeros(rows.value, dtype=np.int32)
    _check(lib.tc_split_terms(h, int(side), terms.ctypes.data_as(ctypes.c_void_p),
                              exps.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                              ctypes.byref(rows), ctypes.byref(kp)))
    return terms, exps


def tc_status_str(s: int) -> str:
    return lib.tc_status_str(int(s)).decode()


def tc_last_error() -> str:
    return lib.tc_last_error().decode(errors="replace")


# ---- convenience wrappers --------------------------------------------------------
def _split(spec):
    out, ins = spec.split("=")
    a, b = ins.split(",")
    return a, b, out


class Plan:
    """A planned contraction.  ``strides`` maps 'A'/'B'/'C' to element strides
    in spec order (missing -> Fortran order)."""

    def __init__(self, spec: str, extents: dict, dtype: str = "f64", strides: dict | None = None,
                 compute: str = "native", products: int | None = None):
        self.spec = spec
        self.extents = dict(extents)
        self.dtype = dtype
        self.letters = _split(spec)
        strides = strides or {}
        self.strides = {t: (list(strides[t]) if t in strides else self._fortran(t)) for t in "ABC"}
        self.handle = tc_plan(spec, self.extents, strides.get("A"), strides.get("B"), strides.get("C"),
                              DTYPES[dtype],
                              dict(native=TC_NATIVE, bf16x3=TC_BF16X3, fp8x3=TC_FP8X3)[compute])
        if products is not None:         # split-BF16 term products: 6, or the ablations 3 and 9
            _check(lib.tc_set_split_products(self.handle, int(products)))

    def _fortran(self, t):
        letters = self.letters["ABC".index(t)]
        st, run = [], 1
        for ch in letters:
            st.append(run)
            run *= self.extents[ch]
        return st

    def shape(self, t):
        return [self.extents[ch] for ch in self.letters["ABC".index(t)]]

    def __del__(self):
        h = getattr(self, "handle", None)
        if h:
            try:
                lib.tc_plan_destroy(h)
            except Exception:
                pass
            self.handle = None

    def variants(self):
        return [tc_variant_get(self.handle, v) for v in range(tc_variant_count(self.handle))]

    def set_variant(self, v):
        tc_set_variant(self.handle, v)

    def prepare(self):
        tc_plan_prepare(self.handle)

    TORCH_DTYPES = dict(f64="float64", f32="float32", c128="complex128", c64="complex64")

    def check_tensors(self, A, B, C, device=True):
        """Raise ValueError unless A, B and C (torch tensors, None where not
        read) are GPU tensors of the plan's dtype, shape and strides (the
        device only with ``device``)."""
        import torch
        want = getattr(torch, self.TORCH_DTYPES[self.dtype])
        for t, x in zip("ABC", (A, B, C)):
            if x is None:
                continue
            if x.dtype != want:
                raise ValueError(f"{t}: dtype {x.dtype} does not match the plan's {self.dtype}")
            if list(x.shape) != self.shape(t) or list(x.stride()) != self.strides[t] and x.numel() > 1:
                raise ValueError(f"{t}: shape/strides {tuple(x.shape)}/{x.stride()} do not match the plan "
                                 f"{self.shape(t)}/{self.strides[t]}")
        for t, x in zip("ABC", (A, B, C) if device else ()):
            if x is not None and not x.is_cuda:
                raise ValueError(f"{t}: tensor on {x.device}, the library takes GPU tensors")

    def contract(self, A, B, C, alpha=1.0, beta=0.0, stream=None):
        """A, B, C: torch tensors on the GPU whose dtype and strides match the plan."""
        import torch
        self.check_tensors(A, B, C)
        if stream is None:
            stream = torch.cuda.current_stream().cuda_stream
        ptrs = [x.data_ptr() if x is not None else 0 for x in (A, B, C)]
        if isinstance(alpha, complex) or isinstance(beta, complex):
            tc_contract_complex(self.handle, *ptrs, alpha, beta, stream)
        else:
            tc_contract(self.handle, *ptrs, alpha, beta, stream)
        return C

    def predict(self):
        return tc_predict(self.handle)

    def set_root_gap(self, gaps=None):
        tc_set_root_gap(self.handle, gaps)

    def bench_classes(self, variant, stage, cache_elems, line_elems):
        return tc_bench_classes(self.handle, variant, stage, cache_elems, line_elems)

    def access_distance(self, variant, tensor):
        return tc_access_distance(self.handle, variant, "ABC".index(tensor) if isinstance(tensor, str) else tensor)


def empty_fortran(shape, dtype, device="cuda"):
    """An uninitialised tensor with Fortran (column-major) strides."""
    import torch
    st, run = [], 1
    for n in shape:
        st.append(run)
        run *= max(1, n)
    return torch.empty_strided(tuple(shape), tuple(st), dtype=dtype, device=device)


def to_device_fortran(x, dtype, device="cuda"):
    """Copy a host numpy array into a Fortran-ordered device tensor (values
    rounded to ``dtype``)."""
    import numpy as np
    import torch
    t = empty_fortran(list(x.shape), dtype, device)
    t.copy_(torch.from_numpy(np.asfortranarray(x)))
    return t
