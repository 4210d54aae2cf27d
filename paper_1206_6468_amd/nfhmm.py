"""Python binding of the C ABI in include/nfhmm.h (ctypes; argument marshalling only).

Every computation runs in libnfhmm.so on the GPU.  Importing this module
raises if the built library is missing; there is no other code path.

Problems are dicts in the ABI layouts (as produced by ``gen.make_problem``):
    V [T][F], W [S][N][K][F], A [S][N][N], pi [S][N], plus gamma, iters and an
    optional alpha_init [T][S*N*K].
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libnfhmm.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(
        f"{LIB_PATH} is missing: build it first (python -c 'import __graft_entry__ as g; g.build()')")
# One HIP runtime per process: when PyTorch is present its bundled runtime must be
# the one libnfhmm.so binds to (same soname), so that device pointers and streams
# created by torch are valid in the library.  Import it before loading the library.
try:
    import torch  # noqa: F401
except ImportError:  # pragma: no cover - the host-pointer API works without torch
    torch = None
_lib = C.CDLL(LIB_PATH)

OK, E_INVALID, E_NOMEM, E_DEVICE, E_NONFINITE, E_CANCELLED, E_NOTFOUND = 0, -1, -2, -3, -4, -5, -6
FP32, BF16 = 0, 1
_STATUS = {0: "OK", -1: "INVALID", -2: "NOMEM", -3: "DEVICE", -4: "NONFINITE", -5: "CANCELLED", -6: "NOTFOUND"}
_PREC = {"fp32": FP32, "bf16": BF16, FP32: FP32, BF16: BF16}

SYMBOLS = [
    "nfhmm_create", "nfhmm_destroy", "nfhmm_last_error", "nfhmm_footprint_bytes",
    "nfhmm_validate", "nfhmm_admission_plan", "nfhmm_fit", "nfhmm_fit_batch",
    "nfhmm_fit_batch_device", "nfhmm_fit_device", "nfhmm_fit_device_noalloc", "nfhmm_submit", "nfhmm_poll",
    "nfhmm_wait", "nfhmm_cancel", "nfhmm_chain_posterior", "nfhmm_special_functions",
    "nfhmm_profile_enable", "nfhmm_profile_read", "nfhmm_profile_select", "nfhmm_set_lanes",
    "nfhmm_stft_frames", "nfhmm_stft", "nfhmm_istft", "nfhmm_stft_device", "nfhmm_istft_device",
    "nfhmm_learn_nhmm", "nfhmm_learn_nhmm_batch", "nfhmm_learn_nhmm_device",
]
K_SPECTRUM, K_COUNTS, K_CHAINS, K_UPDATE, K_POSTERIOR = 0, 1, 2, 3, 4
KERNEL_KINDS = {"spectrum": K_SPECTRUM, "counts": K_COUNTS, "chains": K_CHAINS, "update": K_UPDATE,
                "posterior": K_POSTERIOR}


class nfhmm_problem(C.Structure):
    _fields_ = [("S", C.c_int32), ("N", C.c_int32), ("K", C.c_int32), ("F", C.c_int64),
                ("T", C.c_int64), ("V", C.c_void_p), ("W", C.c_void_p), ("A", C.c_void_p),
                ("pi", C.c_void_p), ("gamma", C.c_float), ("iters", C.c_int32),
                ("alpha_init", C.c_void_p)]


class nfhmm_result(C.Structure):
    _fields_ = [("alpha", C.c_void_p), ("post", C.c_void_p), ("sep", C.c_void_p),
                ("elbo", C.c_void_p)]


class nfhmm_nhmm_problem(C.Structure):
    _fields_ = [("N", C.c_int32), ("K", C.c_int32), ("F", C.c_int64), ("T", C.c_int64),
                ("V", C.c_void_p), ("W", C.c_void_p), ("theta", C.c_void_p), ("A", C.c_void_p),
                ("pi", C.c_void_p), ("iters", C.c_int32)]


class nfhmm_nhmm_result(C.Structure):
    _fields_ = [("W", C.c_void_p), ("theta", C.c_void_p), ("A", C.c_void_p), ("pi", C.c_void_p),
                ("loglik", C.c_void_p)]


_P = C.POINTER
_lib.nfhmm_create.argtypes = [_P(C.c_void_p), C.c_int, C.c_size_t, C.c_int]
_lib.nfhmm_create.restype = C.c_int
_lib.nfhmm_destroy.argtypes = [C.c_void_p]
_lib.nfhmm_destroy.restype = None
_lib.nfhmm_last_error.argtypes = [C.c_void_p]
_lib.nfhmm_last_error.restype = C.c_char_p
_lib.nfhmm_footprint_bytes.argtypes = [_P(nfhmm_problem), C.c_int]
_lib.nfhmm_footprint_bytes.restype = C.c_size_t
_lib.nfhmm_validate.argtypes = [_P(nfhmm_problem), C.c_char_p, C.c_size_t]
_lib.nfhmm_validate.restype = C.c_int
_lib.nfhmm_admission_plan.argtypes = [C.c_int, _P(C.c_size_t), C.c_size_t, C.c_size_t, C.c_int,
                                      C.c_int, _P(C.c_int)]
_lib.nfhmm_admission_plan.restype = C.c_int
for _n in ("nfhmm_fit",):
    getattr(_lib, _n).argtypes = [C.c_void_p, _P(nfhmm_problem), C.c_int, _P(nfhmm_result)]
    getattr(_lib, _n).restype = C.c_int
_lib.nfhmm_fit_batch.argtypes = [C.c_void_p, C.c_int, _P(nfhmm_problem), C.c_int, _P(nfhmm_result)]
_lib.nfhmm_fit_batch.restype = C.c_int
_lib.nfhmm_fit_batch_device.argtypes = [C.c_void_p, C.c_int, _P(nfhmm_problem), C.c_int,
                                        _P(nfhmm_result), C.c_void_p]
_lib.nfhmm_fit_batch_device.restype = C.c_int
_lib.nfhmm_fit_device.argtypes = [C.c_void_p, _P(nfhmm_problem), C.c_int, _P(nfhmm_result), C.c_void_p]
_lib.nfhmm_fit_device.restype = C.c_int
_lib.nfhmm_fit_device_noalloc.argtypes = [C.c_void_p, _P(nfhmm_problem), C.c_int, _P(nfhmm_result), C.c_void_p]
_lib.nfhmm_fit_device_noalloc.restype = C.c_int
_lib.nfhmm_submit.argtypes = [C.c_void_p, _P(nfhmm_problem), C.c_int, _P(nfhmm_result),
                              _P(C.c_uint64)]
_lib.nfhmm_submit.restype = C.c_int
_lib.nfhmm_poll.argtypes = [C.c_void_p, C.c_uint64, _P(C.c_int)]
_lib.nfhmm_poll.restype = C.c_int
_lib.nfhmm_wait.argtypes = [C.c_void_p, C.c_uint64, _P(C.c_double)]
_lib.nfhmm_wait.restype = C.c_int
_lib.nfhmm_cancel.argtypes = [C.c_void_p, C.c_uint64]
_lib.nfhmm_cancel.restype = C.c_int
_lib.nfhmm_chain_posterior.argtypes = [C.c_void_p, C.c_int, C.c_int64, C.c_void_p, C.c_void_p,
                                       C.c_void_p, C.c_void_p, _P(C.c_double)]
_lib.nfhmm_chain_posterior.restype = C.c_int
_lib.nfhmm_special_functions.argtypes = [C.c_void_p, C.c_int64, C.c_void_p, C.c_void_p, C.c_void_p]
_lib.nfhmm_special_functions.restype = C.c_int
_lib.nfhmm_stft_frames.argtypes = [C.c_int32, C.c_int32, C.c_int64]
_lib.nfhmm_stft_frames.restype = C.c_int64
_lib.nfhmm_stft.argtypes = [C.c_void_p, C.c_int32, C.c_int32, C.c_int32, C.c_void_p, C.c_int64, C.c_void_p,
                            C.c_void_p]
_lib.nfhmm_stft.restype = C.c_int
_lib.nfhmm_istft.argtypes = [C.c_void_p, C.c_int32, C.c_int32, C.c_int32, C.c_int32, C.c_void_p, C.c_void_p,
                             C.c_int64, C.c_void_p, C.c_int64]
_lib.nfhmm_istft.restype = C.c_int
_lib.nfhmm_stft_device.argtypes = [C.c_void_p, C.c_int32, C.c_int32, C.c_int32, C.c_void_p, C.c_int64,
                                   C.c_void_p, C.c_void_p, C.c_void_p]
_lib.nfhmm_stft_device.restype = C.c_int
_lib.nfhmm_istft_device.argtypes = [C.c_void_p, C.c_int32, C.c_int32, C.c_int32, C.c_int32, C.c_void_p,
                                    C.c_void_p, C.c_int64, C.c_void_p, C.c_int64, C.c_void_p]
_lib.nfhmm_istft_device.restype = C.c_int
_lib.nfhmm_profile_select.argtypes = [C.c_void_p, C.c_uint]
_lib.nfhmm_set_lanes.argtypes = [C.c_void_p, C.c_int]
_lib.nfhmm_set_lanes.restype = C.c_int
_lib.nfhmm_profile_select.restype = C.c_int
_lib.nfhmm_profile_enable.argtypes = [C.c_void_p, C.c_int]
_lib.nfhmm_profile_enable.restype = C.c_int
_lib.nfhmm_profile_read.argtypes = [C.c_void_p, C.c_int, _P(C.c_int64), _P(C.c_double)]
_lib.nfhmm_profile_read.restype = C.c_int
_lib.nfhmm_learn_nhmm.argtypes = [C.c_void_p, _P(nfhmm_nhmm_problem), _P(nfhmm_nhmm_result)]
_lib.nfhmm_learn_nhmm.restype = C.c_int
_lib.nfhmm_learn_nhmm_batch.argtypes = [C.c_void_p, C.c_int, _P(nfhmm_nhmm_problem), _P(nfhmm_nhmm_result)]
_lib.nfhmm_learn_nhmm_batch.restype = C.c_int
_lib.nfhmm_learn_nhmm_device.argtypes = [C.c_void_p, _P(nfhmm_nhmm_problem), _P(nfhmm_nhmm_result), C.c_void_p]
_lib.nfhmm_learn_nhmm_device.restype = C.c_int


class NfhmmError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"nfhmm status {_STATUS.get(status, status)}: {msg}")
        self.status = status


def _check(st, ctx=None):
    if st != OK:
        raise NfhmmError(st, _lib.nfhmm_last_error(ctx).decode(errors="replace"))


def _f32(x):
    return np.ascontiguousarray(np.asarray(x, dtype=np.float32))


def _ptr(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


class Context:
    """nfhmm_create / nfhmm_destroy."""

    def __init__(self, device: int = 0, hbm_budget_bytes: int = 0, max_slots: int = 64):
        h = C.c_void_p()
        _check(_lib.nfhmm_create(C.byref(h), int(device), int(hbm_budget_bytes), int(max_slots)))
        self.handle = h

    def close(self):
        if getattr(self, "handle", None):
            _lib.nfhmm_destroy(self.handle)
            self.handle = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _problem_struct(prob, keep):
    """Host-memory nfhmm_problem from a problem dict; `keep` holds the arrays alive."""
    S, N, K = int(prob["S"]), int(prob["N"]), int(prob["K"])
    F, T = int(prob["F"]), int(prob["T"])
    V, W, A, pi = (_f32(prob[k]) for k in ("V", "W", "A", "pi"))
    ai = prob.get("alpha_init")
    ai = None if ai is None else _f32(ai)
    keep.extend([V, W, A, pi, ai])
    return nfhmm_problem(S, N, K, F, T, _ptr(V), _ptr(W), _ptr(A), _ptr(pi),
                         float(prob.get("gamma", 1.0)), int(prob["iters"]), _ptr(ai))


OUTPUTS = ("alpha", "post", "sep", "elbo")


def _alloc_outputs(prob, keep, outputs=OUTPUTS, pinned=False):
    """Output arrays of one problem; those not named in `outputs` are skipped (NULL).
    With `pinned` they are views of page-locked host memory (torch's pinned
    allocator), which the library copies into directly."""
    S, N, K, F, T = (int(prob[k]) for k in ("S", "N", "K", "F", "T"))
    it = int(prob["iters"])
    shapes = dict(alpha=((T, S * N * K), np.float32), post=((S, T, N), np.float32),
                  sep=((S, T, F), np.float32), elbo=((max(it, 0),), np.float64))
    if pinned:
        import torch
        tdt = {np.float32: torch.float32, np.float64: torch.float64}
        ts = {k: torch.empty(shapes[k][0], dtype=tdt[shapes[k][1]], pin_memory=True) for k in OUTPUTS if k in outputs}
        keep.append(ts)
        out = {k: t.numpy() for k, t in ts.items()}
    else:
        out = {k: np.empty(*shapes[k]) for k in OUTPUTS if k in outputs}
    keep.append(out)
    return out, nfhmm_result(_ptr(out.get("alpha")), _ptr(out.get("post")), _ptr(out.get("sep")),
                             _ptr(out.get("elbo")) if it > 0 else None)


def footprint_bytes(prob, precision="fp32") -> int:
    keep = []
    return int(_lib.nfhmm_footprint_bytes(C.byref(_problem_struct(prob, keep)), _PREC[precision]))


def validate(prob):
    """Returns (status, message)."""
    keep = []
    buf = C.create_string_buffer(512)
    st = _lib.nfhmm_validate(C.byref(_problem_struct(prob, keep)), buf, 512)
    return st, buf.value.decode()


def admission_plan(footprints, bytes_in_use, budget, resident, max_slots):
    n = len(footprints)
    fp = (C.c_size_t * max(n, 1))(*[int(x) for x in footprints])
    adm = (C.c_int * max(n, 1))()
    k = _lib.nfhmm_admission_plan(n, fp, int(bytes_in_use), int(budget), int(resident), int(max_slots), adm)
    return int(k), [int(adm[i]) for i in range(n)]


def fit(ctx: Context, prob, precision="fp32"):
    """nfhmm_fit on host arrays; returns dict(alpha, post, sep, elbo)."""
    return fit_batch(ctx, [prob], precision)[0]


def fit_batch(ctx: Context, probs, precision="fp32", pinned=False):
    """nfhmm_fit_batch on host arrays; returns one result dict per problem (the
    arrays in pinned host memory with `pinned`)."""
    keep = []
    n = len(probs)
    ps = (nfhmm_problem * n)(*[_problem_struct(p, keep) for p in probs])
    outs, rs = [], []
    for p in probs:
        o, r = _alloc_outputs(p, keep, OUTPUTS, pinned)
        outs.append(o)
        rs.append(r)
    rarr = (nfhmm_result * n)(*rs)
    _check(_lib.nfhmm_fit_batch(ctx.handle, n, ps, _PREC[precision], rarr), ctx.handle)
    return outs   # a pinned array's base is its torch tensor, which keeps the memory


class DeviceJob:
    """Device-resident inputs and outputs of one problem (torch tensors on the GPU)."""

    def __init__(self, prob, device="cuda"):
        import torch
        dev = torch.device(device)
        f = lambda k: torch.as_tensor(_f32(prob[k]), device=dev)  # noqa: E731
        self.S, self.N, self.K = int(prob["S"]), int(prob["N"]), int(prob["K"])
        self.F, self.T, self.iters = int(prob["F"]), int(prob["T"]), int(prob["iters"])
        self.gamma = float(prob.get("gamma", 1.0))
        self.V, self.W, self.A, self.pi = f("V"), f("W"), f("A"), f("pi")
        ai = prob.get("alpha_init")
        self.alpha_init = None if ai is None else torch.as_tensor(_f32(ai), device=dev)
        M = self.S * self.N * self.K
        self.alpha = torch.empty((self.T, M), dtype=torch.float32, device=dev)
        self.post = torch.empty((self.S, self.T, self.N), dtype=torch.float32, device=dev)
        self.sep = torch.empty((self.S, self.T, self.F), dtype=torch.float32, device=dev)
        self.elbo = torch.empty((max(self.iters, 1),), dtype=torch.float64, device=dev)

    def structs(self):
        p = lambda t: None if t is None else C.c_void_p(t.data_ptr())  # noqa: E731
        prob = nfhmm_problem(self.S, self.N, self.K, self.F, self.T, p(self.V), p(self.W), p(self.A),
                             p(self.pi), self.gamma, self.iters, p(self.alpha_init))
        res = nfhmm_result(p(self.alpha), p(self.post), p(self.sep), p(self.elbo) if self.iters > 0 else None)
        return prob, res


def fit_batch_device(ctx: Context, jobs, precision="fp32", stream=None):
    """nfhmm_fit_batch_device on DeviceJob tensors; `stream` is a torch.cuda.Stream or None."""
    n = len(jobs)
    pr = [j.structs() for j in jobs]
    ps = (nfhmm_problem * n)(*[a for a, _ in pr])
    rs = (nfhmm_result * n)(*[b for _, b in pr])
    h = None if stream is None else C.c_void_p(stream.cuda_stream)
    _check(_lib.nfhmm_fit_batch_device(ctx.handle, n, ps, _PREC[precision], rs, h), ctx.handle)


def fit_device(ctx: Context, job, precision="fp32", stream=None):
    fit_batch_device(ctx, [job], precision, stream)


def fit_device_noalloc(ctx: Context, job, precision="fp32", stream=None):
    """nfhmm_fit_device_noalloc on one DeviceJob: the library's fixed working area,
    nothing allocated."""
    prob, res = job.structs()
    h = None if stream is None else C.c_void_p(stream.cuda_stream)
    _check(_lib.nfhmm_fit_device_noalloc(ctx.handle, C.byref(prob), _PREC[precision], C.byref(res), h), ctx.handle)


class Submitted:
    """A job queued with nfhmm_submit; holds its input copies' owner and outputs."""

    def __init__(self, job_id, outputs, keep):
        self.id = job_id
        self.outputs = outputs
        self._keep = keep


def submit(ctx: Context, prob, precision="bf16", outputs=OUTPUTS, pinned=False) -> Submitted:
    """nfhmm_submit; `outputs` names the results to bring back (the others are NULL),
    into pinned host arrays with `pinned`."""
    keep = []
    ps = _problem_struct(prob, keep)
    out, r = _alloc_outputs(prob, keep, outputs, pinned)
    jid = C.c_uint64()
    _check(_lib.nfhmm_submit(ctx.handle, C.byref(ps), _PREC[precision], C.byref(r), C.byref(jid)), ctx.handle)
    return Submitted(int(jid.value), out, keep)


def poll(ctx: Context, job: Submitted) -> bool:
    d = C.c_int()
    _check(_lib.nfhmm_poll(ctx.handle, C.c_uint64(job.id), C.byref(d)), ctx.handle)
    return bool(d.value)


def wait(ctx: Context, job: Submitted):
    """Returns (outputs, latency seconds); raises NfhmmError on a failed job."""
    lat = C.c_double()
    st = _lib.nfhmm_wait(ctx.handle, C.c_uint64(job.id), C.byref(lat))
    _check(st, ctx.handle)
    return job.outputs, float(lat.value)


def wait_status(ctx: Context, job: Submitted):
    """Like wait, but returns (status, outputs, latency) instead of raising."""
    lat = C.c_double()
    st = _lib.nfhmm_wait(ctx.handle, C.c_uint64(job.id), C.byref(lat))
    return int(st), job.outputs, float(lat.value)


def cancel(ctx: Context, job: Submitted):
    _check(_lib.nfhmm_cancel(ctx.handle, C.c_uint64(job.id)), ctx.handle)


def chain_posterior(ctx: Context, logev, A, pi):
    """nfhmm_chain_posterior: marginals [T][N] and ln Z of one chain."""
    lv, A, pi = _f32(logev), _f32(A), _f32(pi)
    T, N = lv.shape
    post = np.empty((T, N), np.float32)
    lnZ = C.c_double()
    _check(_lib.nfhmm_chain_posterior(ctx.handle, N, T, _ptr(lv), _ptr(A), _ptr(pi), _ptr(post),
                                      C.byref(lnZ)), ctx.handle)
    return post, float(lnZ.value)


def special_functions(ctx: Context, x):
    """nfhmm_special_functions: device digamma and log-gamma of x (float32)."""
    x = _f32(x).ravel()
    psi, lg = np.empty_like(x), np.empty_like(x)
    _check(_lib.nfhmm_special_functions(ctx.handle, x.size, _ptr(x), _ptr(psi), _ptr(lg)), ctx.handle)
    return psi, lg


def stft_frames(nfft: int, hop: int, n: int) -> int:
    """nfhmm_stft_frames: frames of a signal of n samples."""
    return int(_lib.nfhmm_stft_frames(int(nfft), int(hop), int(n)))


def stft(ctx: Context, x, nfft=1024, hop=256):
    """nfhmm_stft on host arrays: x [n] or [B][n] -> (mag, phase), each [B][T][nfft/2+1]
    (the leading B dropped for a 1-d x)."""
    x = _f32(x)
    one = x.ndim == 1
    x2 = x.reshape(1, -1) if one else x
    B, n = x2.shape
    T = stft_frames(nfft, hop, n)
    mag = np.empty((B, max(T, 0), nfft // 2 + 1), dtype=np.float32)
    phase = np.empty_like(mag)
    _check(_lib.nfhmm_stft(ctx.handle, nfft, hop, B, _ptr(x2), n, _ptr(mag), _ptr(phase)), ctx.handle)
    return (mag[0], phase[0]) if one else (mag, phase)


def istft(ctx: Context, mag, phase, n, nfft=1024, hop=256):
    """nfhmm_istft on host arrays.  mag [T][F] with phase [T][F] -> y [n]; mag [S][T][F]
    (S sources of one mixture) with phase [T][F] -> y [S][n]; mag [B][S][T][F] with
    phase [B][T][F] -> y [B][S][n]."""
    mag, phase = _f32(mag), _f32(phase)
    m4 = mag.reshape((1, 1) + mag.shape) if mag.ndim == 2 else mag.reshape((1,) + mag.shape) if mag.ndim == 3 \
        else mag
    B, S, T, F = m4.shape
    # one phase per mixture: [T][F] only when there is one mixture
    if phase.shape != (B, T, F) and not (B == 1 and phase.shape == (T, F)):
        raise ValueError(f"phase shape {phase.shape} does not match mag {mag.shape} (want {(B, T, F)})")
    y = np.empty((B, S, int(n)), dtype=np.float32)
    _check(_lib.nfhmm_istft(ctx.handle, nfft, hop, B, S, _ptr(m4), _ptr(phase), T, _ptr(y), int(n)), ctx.handle)
    return y.reshape(mag.shape[:-2] + (int(n),))


def _dev_f32(t, shape, name):
    import torch
    if t.dtype != torch.float32 or not t.is_cuda or not t.is_contiguous() or tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name}: want a contiguous float32 cuda tensor of shape {tuple(shape)}, "
                         f"got {t.dtype} {tuple(t.shape)} on {t.device}")
    return C.c_void_p(t.data_ptr())


def stft_device(ctx: Context, x, mag, phase, nfft=1024, hop=256, stream=None):
    """nfhmm_stft_device on torch tensors: x [B][n], mag / phase [B][T][nfft/2+1] (float32, cuda)."""
    B, n = x.shape
    shp = (B, stft_frames(nfft, hop, n), nfft // 2 + 1)
    h = None if stream is None else C.c_void_p(stream.cuda_stream)
    _check(_lib.nfhmm_stft_device(ctx.handle, nfft, hop, B, _dev_f32(x, (B, n), "x"), n,
                                  _dev_f32(mag, shp, "mag"), _dev_f32(phase, shp, "phase"), h), ctx.handle)


def istft_device(ctx: Context, mag, phase, y, nfft=1024, hop=256, stream=None):
    """nfhmm_istft_device on torch tensors: mag [B][S][T][F], phase [B][T][F], y [B][S][n]."""
    B, S, T, F = mag.shape
    n = y.shape[-1]
    h = None if stream is None else C.c_void_p(stream.cuda_stream)
    _check(_lib.nfhmm_istft_device(ctx.handle, nfft, hop, B, S, _dev_f32(mag, (B, S, T, nfft // 2 + 1), "mag"),
                                   _dev_f32(phase, (B, T, F), "phase"), T, _dev_f32(y, (B, S, n), "y"), n, h),
           ctx.handle)


def profile_enable(ctx: Context, enable: bool = True):
    """nfhmm_profile_enable: time every later iteration launch with HIP events."""
    _check(_lib.nfhmm_profile_enable(ctx.handle, 1 if enable else 0), ctx.handle)


def set_lanes(ctx: Context, lanes: int):
    """nfhmm_set_lanes: stream lanes a blocking batch is split across (1 or 2)."""
    _check(_lib.nfhmm_set_lanes(ctx.handle, int(lanes)), ctx.handle)


def profile_select(ctx: Context, kinds=None):
    """nfhmm_profile_select: time only these kernel kinds (None: every kind)."""
    mask = 0xFFFFFFFF if kinds is None else sum(1 << KERNEL_KINDS.get(k, k) for k in kinds)
    _check(_lib.nfhmm_profile_select(ctx.handle, C.c_uint(mask)), ctx.handle)


def profile_read(ctx: Context, kind):
    """nfhmm_profile_read: (launches, total device milliseconds) of one kernel kind."""
    n, ms = C.c_int64(), C.c_double()
    _check(_lib.nfhmm_profile_read(ctx.handle, KERNEL_KINDS.get(kind, kind), C.byref(n), C.byref(ms)), ctx.handle)
    return int(n.value), float(ms.value)


def _nhmm_structs(prob, iters, keep):
    """Host nfhmm_nhmm_problem / result and the output dict of one EM problem."""
    V, W, th, A, pi = (_f32(prob[k]) for k in ("V", "W", "theta", "A", "pi"))
    T, F = V.shape
    N, K = W.shape[0], W.shape[1]
    it = int(prob["iters"] if iters is None else iters)
    out = dict(W=np.empty_like(W), theta=np.empty_like(th), A=np.empty_like(A), pi=np.empty_like(pi),
               loglik=np.empty(it, np.float64))
    keep.extend([V, W, th, A, pi])
    p = nfhmm_nhmm_problem(N, K, F, T, _ptr(V), _ptr(W), _ptr(th), _ptr(A), _ptr(pi), it)
    r = nfhmm_nhmm_result(*(_ptr(out[k]) for k in ("W", "theta", "A", "pi", "loglik")))
    return p, r, out


def learn_nhmm(ctx: Context, prob, iters=None):
    """nfhmm_learn_nhmm on host arrays.  prob: V [T][F], W [N][K][F], theta [T][N][K],
    A [N][N], pi [N] (the starting parameters) and iters; returns dict(W, theta, A, pi,
    loglik)."""
    keep = []
    p, r, out = _nhmm_structs(prob, iters, keep)
    _check(_lib.nfhmm_learn_nhmm(ctx.handle, C.byref(p), C.byref(r)), ctx.handle)
    return out


def learn_nhmm_batch(ctx: Context, probs, iters=None):
    """nfhmm_learn_nhmm_batch on host arrays: one result dict per problem."""
    keep = []
    st = [_nhmm_structs(q, iters, keep) for q in probs]
    n = len(st)
    ps = (nfhmm_nhmm_problem * n)(*[a for a, _, _ in st])
    rs = (nfhmm_nhmm_result * n)(*[b for _, b, _ in st])
    _check(_lib.nfhmm_learn_nhmm_batch(ctx.handle, n, ps, rs), ctx.handle)
    return [o for _, _, o in st]


class DeviceNhmm:
    """Device-resident inputs and outputs of one EM problem (torch tensors on the GPU)."""

    def __init__(self, prob, iters=None, device="cuda"):
        import torch
        dev = torch.device(device)
        f = lambda k: torch.as_tensor(_f32(prob[k]), device=dev)  # noqa: E731
        self.V, self.W, self.theta, self.A, self.pi = (f(k) for k in ("V", "W", "theta", "A", "pi"))
        self.T, self.F = self.V.shape
        self.N, self.K = self.W.shape[0], self.W.shape[1]
        self.iters = int(prob["iters"] if iters is None else iters)
        self.W_out, self.theta_out = torch.empty_like(self.W), torch.empty_like(self.theta)
        self.A_out, self.pi_out = torch.empty_like(self.A), torch.empty_like(self.pi)
        self.loglik = torch.empty((self.iters,), dtype=torch.float64, device=dev)

    def structs(self):
        p = lambda t: C.c_void_p(t.data_ptr())  # noqa: E731
        prob = nfhmm_nhmm_problem(self.N, self.K, self.F, self.T, p(self.V), p(self.W), p(self.theta), p(self.A),
                                  p(self.pi), self.iters)
        res = nfhmm_nhmm_result(p(self.W_out), p(self.theta_out), p(self.A_out), p(self.pi_out), p(self.loglik))
        return prob, res


def learn_nhmm_device(ctx: Context, job: DeviceNhmm, stream=None):
    """nfhmm_learn_nhmm_device on DeviceNhmm tensors."""
    prob, res = job.structs()
    h = None if stream is None else C.c_void_p(stream.cuda_stream)
    _check(_lib.nfhmm_learn_nhmm_device(ctx.handle, C.byref(prob), C.byref(res), h), ctx.handle)
