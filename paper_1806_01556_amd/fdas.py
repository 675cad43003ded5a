"""Thin ctypes binding of libfdas (the C ABI in include/fdas.h).

Argument marshalling only: every step of the hot path runs in the library's
HIP kernels.  Device buffers are torch tensors (or raw integer device
addresses); streams are torch streams or raw hipStream_t integers.  If the
shared library is not built this module raises on first use -- there is no
fallback path.
"""

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libfdas.so")

# status codes
OK, ERR_INVALID_ARG, ERR_NO_DEVICE, ERR_OUT_OF_MEMORY, ERR_DEVICE, ERR_CAPACITY, ERR_UNSUPPORTED = range(7)
STATUS_NAMES = {
    0: "FDAS_OK", 1: "FDAS_ERR_INVALID_ARG", 2: "FDAS_ERR_NO_DEVICE", 3: "FDAS_ERR_OUT_OF_MEMORY",
    4: "FDAS_ERR_DEVICE", 5: "FDAS_ERR_CAPACITY", 6: "FDAS_ERR_UNSUPPORTED",
}
CONV_AUTO, CONV_OLS_FFT, CONV_DIRECT_MFMA = 0, 1, 2
PREC_FP32, PREC_SPLIT_FP16, PREC_SPLIT_BF16 = 0, 1, 2
HSUM_STRETCH, HSUM_FUNDAMENTAL, HSUM_HIGHEST = 0, 1, 2

#: symbols declared in include/fdas.h
EXPORTED = (
    "fdas_plan_desc_default", "fdas_plan_create", "fdas_plan_destroy", "fdas_convolve",
    "fdas_harmonic_sum", "fdas_candidates", "fdas_last_error", "fdas_abi_version",
    "fdas_template_taps", "fdas_thresholds", "fdas_search_batch", "fdas_candidates_batch",
    "fdas_autotune", "fdas_set_tuning", "fdas_candidates_mapped", "fdas_prescreen_param_count",
    "fdas_prescreen_create", "fdas_prescreen_destroy", "fdas_prescreen_set_params", "fdas_prescreen_get_params",
    "fdas_prescreen_features", "fdas_prescreen_forward", "fdas_prescreen_infer", "fdas_prescreen_gradient",
    "fdas_prescreen_train_step", "fdas_search_blocks", "fdas_search_flagged", "fdas_block_closure",
    "fdas_prescreen_init_params", "fdas_harmonic_sum_noalloc",
)


class PlanDesc(ctypes.Structure):
    _fields_ = [
        ("struct_size", ctypes.c_int32),
        ("n_max", ctypes.c_int64),
        ("z_max", ctypes.c_int32),
        ("n_harm", ctypes.c_int32),
        ("p_fa", ctypes.c_double),
        ("cand_capacity", ctypes.c_int32),
        ("top_k", ctypes.c_int32),
        ("method", ctypes.c_int32),
        ("precision", ctypes.c_int32),
        ("hsum_index", ctypes.c_int32),
        ("ols_chunk", ctypes.c_int32),
        ("device", ctypes.c_int32),
    ]


class Cand(ctypes.Structure):
    _fields_ = [("harm", ctypes.c_int32), ("z", ctypes.c_int32), ("r", ctypes.c_int32), ("power", ctypes.c_float)]


class Trial(ctypes.Structure):
    _fields_ = [
        ("d_spectrum", ctypes.c_void_p),
        ("n", ctypes.c_int64),
        ("d_fop", ctypes.c_void_p),
        ("ld", ctypes.c_int64),
        ("d_cands", ctypes.c_void_p),
        ("d_counts", ctypes.c_void_p),
    ]


class Tuning(ctypes.Structure):
    _fields_ = [
        ("conv_templates_per_item", ctypes.c_int32),
        ("conv_waves_per_simd", ctypes.c_int32),
        ("overlap_groups", ctypes.c_int32),
        ("emit_workgroups", ctypes.c_int32),
        ("ols_chunk", ctypes.c_int32),
        ("hsum_tile", ctypes.c_int32),
    ]

    def as_dict(self):
        return {f: int(getattr(self, f)) for f, _ in self._fields_}


CAND_DTYPE = np.dtype([("harm", np.int32), ("z", np.int32), ("r", np.int32), ("power", np.float32)])


class FdasError(RuntimeError):
    def __init__(self, status, message):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {message}")
        self.status = status


_lib = None


def lib():
    """The loaded libfdas (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built; run `python -m paper_1806_01556_amd.build`")
    L = ctypes.CDLL(LIB_PATH)
    vp, i32, i64, dbl = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    L.fdas_plan_desc_default.argtypes = [ctypes.POINTER(PlanDesc)]
    L.fdas_plan_desc_default.restype = None
    L.fdas_plan_create.argtypes = [ctypes.POINTER(PlanDesc), ctypes.POINTER(vp)]
    L.fdas_plan_destroy.argtypes = [vp]
    L.fdas_convolve.argtypes = [vp, vp, i64, vp, i64, vp]
    L.fdas_harmonic_sum.argtypes = [vp, vp, i64, i64, vp, vp, vp, vp]
    L.fdas_harmonic_sum_noalloc.argtypes = [vp, vp, i64, i64, vp, vp, vp, vp]
    L.fdas_candidates.argtypes = [vp, vp, vp, vp, i64, ctypes.POINTER(i64), vp, vp]
    L.fdas_last_error.argtypes = []
    L.fdas_last_error.restype = ctypes.c_char_p
    L.fdas_abi_version.argtypes = []
    L.fdas_abi_version.restype = i32
    L.fdas_template_taps.argtypes = [i32, vp, i32, ctypes.POINTER(i32)]
    L.fdas_thresholds.argtypes = [i32, dbl, vp]
    L.fdas_search_batch.argtypes = [vp, ctypes.POINTER(Trial), i32, vp]
    L.fdas_candidates_batch.argtypes = [vp, ctypes.POINTER(Trial), i32, vp, i64, vp, vp, vp]
    L.fdas_autotune.argtypes = [vp, ctypes.POINTER(Trial), i32, i32, ctypes.POINTER(Tuning), vp]
    L.fdas_set_tuning.argtypes = [vp, ctypes.POINTER(Tuning)]
    L.fdas_candidates_mapped.argtypes = [vp, vp, vp, ctypes.POINTER(vp), ctypes.POINTER(i64), vp, vp]
    flt = ctypes.c_float
    L.fdas_prescreen_param_count.argtypes = []
    L.fdas_prescreen_param_count.restype = i32
    L.fdas_prescreen_create.argtypes = [i32, i32, ctypes.POINTER(vp)]
    L.fdas_prescreen_destroy.argtypes = [vp]
    L.fdas_prescreen_set_params.argtypes = [vp, vp]
    L.fdas_prescreen_get_params.argtypes = [vp, vp]
    L.fdas_prescreen_features.argtypes = [vp, vp, i64, vp, i32, vp, vp]
    L.fdas_prescreen_forward.argtypes = [vp, vp, i32, vp, vp]
    L.fdas_prescreen_infer.argtypes = [vp, vp, i64, i32, vp, vp]
    L.fdas_prescreen_gradient.argtypes = [vp, vp, vp, i32, flt, vp, vp, vp, vp]
    L.fdas_prescreen_train_step.argtypes = [vp, vp, vp, i32, flt, flt, vp, vp, vp]
    L.fdas_search_blocks.argtypes = [vp, vp, i64, vp, i64, vp, i32, vp, vp, vp]
    L.fdas_search_flagged.argtypes = [vp, vp, i64, vp, i64, vp, ctypes.c_float, vp, vp, vp]
    L.fdas_block_closure.argtypes = [i64, i32, vp, i32, vp, i32, ctypes.POINTER(i32)]
    L.fdas_prescreen_init_params.argtypes = [ctypes.c_uint64, vp]
    for name in ("fdas_plan_create", "fdas_plan_destroy", "fdas_convolve", "fdas_harmonic_sum",
                 "fdas_candidates", "fdas_template_taps", "fdas_thresholds", "fdas_search_batch",
                 "fdas_candidates_batch", "fdas_autotune", "fdas_set_tuning", "fdas_candidates_mapped",
                 "fdas_prescreen_create", "fdas_prescreen_destroy", "fdas_prescreen_set_params",
                 "fdas_prescreen_get_params", "fdas_prescreen_features", "fdas_prescreen_forward",
                 "fdas_prescreen_infer", "fdas_prescreen_gradient", "fdas_prescreen_train_step", "fdas_search_blocks",
                 "fdas_search_flagged", "fdas_block_closure", "fdas_prescreen_init_params",
                 "fdas_harmonic_sum_noalloc"):
        getattr(L, name).restype = ctypes.c_int
    _lib = L
    return L


def last_error():
    return lib().fdas_last_error().decode()


def _check(status):
    if status != OK:
        raise FdasError(status, last_error())


def _ptr(x):
    """Device/host address of a torch tensor, numpy array or integer (None -> NULL)."""
    if x is None:
        return None
    if isinstance(x, int):
        return x
    if hasattr(x, "data_ptr"):
        return x.data_ptr()
    if isinstance(x, np.ndarray):
        return x.ctypes.data
    raise TypeError(f"cannot take the address of {type(x)}")


def _stream(s):
    if s is None:
        try:
            import torch
            if torch.cuda.is_available():
                return torch.cuda.current_stream().cuda_stream
        except ImportError:
            pass
        return None
    if isinstance(s, int):
        return s
    return s.cuda_stream


def abi_version():
    return lib().fdas_abi_version()


def plan_desc_default(**overrides):
    d = PlanDesc()
    lib().fdas_plan_desc_default(ctypes.byref(d))
    for k, v in overrides.items():
        if not hasattr(d, k):
            raise AttributeError(k)
        setattr(d, k, v)
    return d


class Plan:
    """Owns an fdas_plan*; destroy() (or the context manager) releases it."""

    def __init__(self, handle, desc):
        self.handle = handle
        self.desc = desc
        self.rows = 2 * desc.z_max + 1
        self._host_out = None  # pinned candidate buffer, allocated on first use

    def destroy(self):
        if self.handle:
            _check(lib().fdas_plan_destroy(self.handle))
            self.handle = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.destroy()


def plan_create(desc=None, **overrides):
    if desc is None:
        desc = plan_desc_default(**overrides)
    h = ctypes.c_void_p()
    _check(lib().fdas_plan_create(ctypes.byref(desc), ctypes.byref(h)))
    return Plan(h.value, desc)


def plan_destroy(plan):
    plan.destroy()


def convolve(plan, spectrum, fop, n=None, ld=None, stream=None):
    """FOP[z + z_max, j] = |sum_d X[j+d] h_z[d]|^2 for j < n (asynchronous)."""
    if n is None:
        n = spectrum.shape[0]
    if ld is None:
        ld = fop.shape[1] if hasattr(fop, "shape") and len(fop.shape) == 2 else n
    _check(lib().fdas_convolve(plan.handle, _ptr(spectrum), int(n), _ptr(fop), int(ld), _stream(stream)))


def harmonic_sum(plan, fop, n, cands, counts, ta=None, ld=None, stream=None):
    """Algorithm 1 over the FOP; appends cells above TA to cands, counts per plane (asynchronous)."""
    if ld is None:
        ld = fop.shape[1]
    _check(lib().fdas_harmonic_sum(plan.handle, _ptr(fop), int(n), int(ld), _ptr(ta), _ptr(cands),
                                   _ptr(counts), _stream(stream)))


def harmonic_sum_noalloc(plan, fop, n, cands, counts, ta=None, ld=None, stream=None):
    """fdas_harmonic_sum with its scratch in the library's static device array
    (allocates nothing; n <= 2^22; asynchronous)."""
    if ld is None:
        ld = fop.shape[1]
    _check(lib().fdas_harmonic_sum_noalloc(plan.handle, _ptr(fop), int(n), int(ld), _ptr(ta), _ptr(cands),
                                           _ptr(counts), _stream(stream)))


def _pinned_out(plan, capacity):
    """Reusable page-locked host buffer of `capacity` records (numpy view)."""
    buf = plan._host_out
    if buf is None or buf[1].shape[0] < capacity:
        try:
            import torch
            t = torch.empty((capacity * CAND_DTYPE.itemsize,), dtype=torch.uint8, pin_memory=True)
            arr = t.numpy().view(CAND_DTYPE)
        except Exception:
            t, arr = None, np.empty(capacity, dtype=CAND_DTYPE)
        plan._host_out = buf = (t, arr)
    return buf[1]


def candidates(plan, cands, counts, capacity=None, stream=None, allow_overflow=False, copy=True):
    """Ordered candidate records (numpy CAND_DTYPE) and the per-plane device counts.

    The library orders the lists on the device.  Without a capacity the
    records are written by the device into a page-locked buffer owned by the
    plan (fdas_candidates_mapped); with copy=False the returned array is a
    view of that buffer, overwritten by the plan's next readback.  With a
    capacity the copying call fdas_candidates is used.
    """
    nh = plan.desc.n_harm
    hc = np.zeros(nh, dtype=np.int32)
    nw = ctypes.c_int64(0)
    if capacity is None:
        view = ctypes.c_void_p()
        st = lib().fdas_candidates_mapped(plan.handle, _ptr(cands), _ptr(counts), ctypes.byref(view),
                                          ctypes.byref(nw), hc.ctypes.data, _stream(stream))
        if not (st == ERR_CAPACITY and allow_overflow):
            _check(st)
        if nw.value == 0 or not view.value:
            return np.empty(0, dtype=CAND_DTYPE), hc
        buf = (ctypes.c_char * (nw.value * CAND_DTYPE.itemsize)).from_address(view.value)
        res = np.frombuffer(buf, dtype=CAND_DTYPE, count=nw.value)
        return (res.copy() if copy else res), hc
    out = _pinned_out(plan, capacity)
    st = lib().fdas_candidates(plan.handle, _ptr(cands), _ptr(counts), out.ctypes.data, int(capacity),
                               ctypes.byref(nw), hc.ctypes.data, _stream(stream))
    if not (st == ERR_CAPACITY and allow_overflow):
        _check(st)
    res = out[: nw.value]
    return (res.copy() if copy else res), hc


def template_taps(z):
    """FP64 taps of template z as complex128[L] (offsets -L/2 .. L/2-1)."""
    n = ctypes.c_int32(0)
    lib().fdas_template_taps(int(z), None, 0, ctypes.byref(n))
    buf = np.zeros(2 * n.value, dtype=np.float64)
    _check(lib().fdas_template_taps(int(z), buf.ctypes.data, n.value, ctypes.byref(n)))
    return buf[0::2] + 1j * buf[1::2]


def thresholds(n_harm=8, p_fa=1e-6):
    out = np.zeros(n_harm, dtype=np.float64)
    _check(lib().fdas_thresholds(int(n_harm), float(p_fa), out.ctypes.data))
    return out


# ---- batches of dispersion trials ---------------------------------------------

def trials_array(items):
    """ctypes array of Trial from (spectrum, n, fop, ld, cands, counts) tuples
    (torch tensors or integer device addresses)."""
    arr = (Trial * len(items))()
    for t, (x, n, fop, ld, cands, counts) in zip(arr, items):
        t.d_spectrum, t.n, t.d_fop, t.ld = _ptr(x), int(n), _ptr(fop), int(ld)
        t.d_cands, t.d_counts = _ptr(cands), _ptr(counts)
    return arr


def search_batch(plan, trials, stream=None):
    """Convolution + harmonic sum of every trial (asynchronous; a Trial array)."""
    _check(lib().fdas_search_batch(plan.handle, trials, len(trials), _stream(stream)))


def candidates_batch(plan, trials, capacity=None, stream=None, allow_overflow=False, copy=True):
    """Ordered candidates of every trial: (list of CAND_DTYPE arrays, counts[count][n_harm]).

    With copy=False the arrays are views of the plan's page-locked buffer,
    overwritten by the plan's next readback."""
    count, nh = len(trials), plan.desc.n_harm
    if capacity is None:
        capacity = count * nh * plan.desc.cand_capacity if plan.desc.top_k <= 0 else count * nh * plan.desc.top_k
    out = _pinned_out(plan, capacity)
    offs = np.zeros(count + 1, dtype=np.int64)
    hc = np.zeros((count, nh), dtype=np.int32)
    st = lib().fdas_candidates_batch(plan.handle, trials, count, out.ctypes.data, int(capacity), offs.ctypes.data,
                                     hc.ctypes.data, _stream(stream))
    if not (st == ERR_CAPACITY and allow_overflow):
        _check(st)
    views = [out[offs[i]:offs[i + 1]] for i in range(count)]
    return ([v.copy() for v in views] if copy else views), hc


def autotune(plan, trials, repeats=3, stream=None):
    """Time the batch path over its launch parameters; the fastest is kept in the plan (returned as a dict)."""
    t = Tuning()
    _check(lib().fdas_autotune(plan.handle, trials, len(trials), int(repeats), ctypes.byref(t), _stream(stream)))
    return t.as_dict()


def set_tuning(plan, **fields):
    """Set batch launch parameters by hand (no fields: defaults)."""
    t = Tuning()
    for k, v in fields.items():
        setattr(t, k, int(v))
    _check(lib().fdas_set_tuning(plan.handle, ctypes.byref(t) if fields else None))


# ---- learned block pre-screen --------------------------------------------------

BLOCK = 4096


class Prescreen:
    """Owns an fdas_prescreen* (network parameters, Adam state, workspace)."""

    def __init__(self, max_batch=256, device=0):
        h = ctypes.c_void_p()
        _check(lib().fdas_prescreen_create(int(device), int(max_batch), ctypes.byref(h)))
        self.handle = h.value
        self.max_batch = int(max_batch)

    @staticmethod
    def param_count():
        return int(lib().fdas_prescreen_param_count())

    def destroy(self):
        if self.handle:
            _check(lib().fdas_prescreen_destroy(self.handle))
            self.handle = None

    def set_params(self, theta):
        theta = np.ascontiguousarray(theta, dtype=np.float32)
        assert theta.size == self.param_count()
        _check(lib().fdas_prescreen_set_params(self.handle, theta.ctypes.data))

    def get_params(self):
        out = np.zeros(self.param_count(), dtype=np.float32)
        _check(lib().fdas_prescreen_get_params(self.handle, out.ctypes.data))
        return out

    def features(self, spectrum, n, blocks, out, stream=None):
        """Features of the listed blocks; an int `blocks` means blocks 0 .. blocks-1 (no host list)."""
        if isinstance(blocks, (int, np.integer)):
            _check(lib().fdas_prescreen_features(self.handle, _ptr(spectrum), int(n), None, int(blocks), _ptr(out),
                                                 _stream(stream)))
            return
        blocks = np.ascontiguousarray(blocks, dtype=np.int32)
        _check(lib().fdas_prescreen_features(self.handle, _ptr(spectrum), int(n), blocks.ctypes.data, blocks.size,
                                             _ptr(out), _stream(stream)))

    def forward(self, feats, nb, logits, stream=None):
        _check(lib().fdas_prescreen_forward(self.handle, _ptr(feats), int(nb), _ptr(logits), _stream(stream)))

    def infer(self, spectrum, n, nb, logits, stream=None):
        """Logits of blocks 0 .. nb-1 straight from the spectrum (features computed in the kernel)."""
        _check(lib().fdas_prescreen_infer(self.handle, _ptr(spectrum), int(n), int(nb), _ptr(logits),
                                          _stream(stream)))

    def gradient(self, feats, labels, nb, pos_weight, logits, loss, grad=None, stream=None):
        _check(lib().fdas_prescreen_gradient(self.handle, _ptr(feats), _ptr(labels), int(nb), float(pos_weight),
                                             _ptr(logits), _ptr(loss), _ptr(grad), _stream(stream)))

    def train_step(self, feats, labels, nb, pos_weight, lr, logits, loss, stream=None):
        _check(lib().fdas_prescreen_train_step(self.handle, _ptr(feats), _ptr(labels), int(nb), float(pos_weight),
                                               float(lr), _ptr(logits), _ptr(loss), _stream(stream)))


def prescreen_init_params(seed=0):
    """Initial network parameters from the library (float32[param_count])."""
    out = np.zeros(int(lib().fdas_prescreen_param_count()), dtype=np.float32)
    _check(lib().fdas_prescreen_init_params(int(seed), out.ctypes.data))
    return out


def search_blocks(plan, spectrum, n, fop, blocks, cands, counts, ld=None, stream=None):
    """The two-step search on the listed 4096-bin blocks only (asynchronous)."""
    if ld is None:
        ld = fop.shape[1]
    blocks = np.ascontiguousarray(blocks, dtype=np.int32)
    _check(lib().fdas_search_blocks(plan.handle, _ptr(spectrum), int(n), _ptr(fop), int(ld), blocks.ctypes.data,
                                    blocks.size, _ptr(cands), _ptr(counts), _stream(stream)))


def search_flagged(plan, spectrum, n, fop, logits, threshold, cands, counts, ld=None, stream=None):
    """The restricted search on the blocks whose logit exceeds threshold, plus
    their harmonic closure, selected on the device (asynchronous).  logits None
    (screen disabled), a non-finite logit or a NaN threshold search every block."""
    if ld is None:
        ld = fop.shape[1]
    _check(lib().fdas_search_flagged(plan.handle, _ptr(spectrum), int(n), _ptr(fop), int(ld), _ptr(logits),
                                     float(threshold), _ptr(cands), _ptr(counts), _stream(stream)))


def block_closure(blocks, n, n_harm=8):
    """The library's harmonic closure of a block list (sorted int32 array)."""
    blocks = np.ascontiguousarray(blocks, dtype=np.int32)
    cap = (int(n) + BLOCK - 1) // BLOCK
    out = np.zeros(max(cap, 1), dtype=np.int32)
    cnt = ctypes.c_int32(0)
    _check(lib().fdas_block_closure(int(n), int(n_harm), blocks.ctypes.data if blocks.size else None, blocks.size,
                                    out.ctypes.data, cap, ctypes.byref(cnt)))
    return out[:cnt.value].copy()


# ---- torch conveniences ------------------------------------------------------

def fop_ld(n):
    """Row stride used by the helpers: n rounded up to a multiple of 64 floats."""
    return (int(n) + 63) // 64 * 64


def alloc_fop(plan, n, device="cuda"):
    import torch
    return torch.empty((plan.rows, fop_ld(n)), dtype=torch.float32, device=device)


def alloc_cands(plan, device="cuda"):
    import torch
    nh, cap = plan.desc.n_harm, plan.desc.cand_capacity
    cands = torch.empty((nh * cap * 4,), dtype=torch.int32, device=device)
    counts = torch.zeros((nh,), dtype=torch.int32, device=device)
    return cands, counts


def search(plan, spectrum, fop=None, cands=None, counts=None, stream=None):
    """Both hot-path steps and the readback: (ordered candidates, counts, fop)."""
    n = spectrum.shape[0]
    if fop is None:
        fop = alloc_fop(plan, n, spectrum.device)
    if cands is None:
        cands, counts = alloc_cands(plan, spectrum.device)
    convolve(plan, spectrum, fop, n=n, stream=stream)
    harmonic_sum(plan, fop, n, cands, counts, stream=stream)
    c, hc = candidates(plan, cands, counts, stream=stream, allow_overflow=True)
    return c, hc, fop
