"""Host-side checks of the C-ABI library: it loads, exports every declared
symbol, and its host-only entry points (validation, footprint, admission)
behave as documented.  No device is used."""
import ctypes
import os
import re

import numpy as np
import pytest

from gen import make_problem, make_tiny

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "nfhmm.h")).read()
    return sorted(set(re.findall(r"NFHMM_API\s+[\w\s\*]+?\b(nfhmm_\w+)\s*\(", src)))


@pytest.fixture(scope="module")
def L():
    from paper_1206_6468_amd import nfhmm
    return nfhmm


def test_library_exports_every_declared_symbol(L):
    decl = _declared()
    assert len(decl) >= 16
    lib = ctypes.CDLL(L.LIB_PATH)
    for name in decl:
        assert hasattr(lib, name), name
    assert sorted(L.SYMBOLS) == decl


def test_validate_accepts_generated_problems(L):
    for p in (make_problem(0, 0), make_tiny()):
        st, msg = L.validate(p)
        assert st == L.OK, msg


@pytest.mark.parametrize("mutate,needle", [
    (lambda p: p["V"].__setitem__((0, 0), np.nan), "V["),
    (lambda p: p["V"].__setitem__((1, 2), -1.0), "V["),
    (lambda p: p["W"].__setitem__((0, 0, 0, 0), p["W"][0, 0, 0, 0] + 0.01), "sums to"),
    (lambda p: p["A"].__setitem__((0, 0, 0), p["A"][0, 0, 0] + 0.01), "row"),
    (lambda p: p["pi"].__setitem__((1, 0), p["pi"][1, 0] + 0.01), "pi"),
])
def test_validate_rejects(L, mutate, needle):
    p = make_tiny()
    p = {k: (v.copy() if isinstance(v, np.ndarray) else v) for k, v in p.items()}
    mutate(p)
    st, msg = L.validate(p)
    assert st == L.E_INVALID and needle in msg, msg


def test_validate_rejects_unexplainable_bin(L):
    p = make_tiny(F=6)
    p = {k: (v.copy() if isinstance(v, np.ndarray) else v) for k, v in p.items()}
    W = p["W"].astype(np.float64)
    W[..., 2] = 0.0
    W /= W.sum(-1, keepdims=True)
    p["W"] = W.astype(np.float32)
    p["V"][0, 2] = 3.0
    st, msg = L.validate(p)
    assert st == L.E_INVALID and "bin 2" in msg


@pytest.mark.parametrize("over,needle", [
    (dict(S=0), "S out of range"), (dict(N=65), "N out of range"), (dict(K=0), "K must"),
    (dict(iters=-1), "iters"), (dict(gamma=-1.0), "gamma"),
])
def test_validate_rejects_dims(L, over, needle):
    p = dict(make_tiny(), **over)
    st, msg = L.validate(p)
    assert st == L.E_INVALID and needle in msg, msg


def test_footprint_grows_with_shape(L):
    a = L.footprint_bytes(make_problem(0, 0))
    b = L.footprint_bytes(make_problem(1, 0))
    c = L.footprint_bytes(make_problem(1, 0), "bf16")
    assert 0 < a < b
    # bf16 keeps extra operand copies but drops the float32 w and R
    assert c != b
    assert L.footprint_bytes(dict(make_tiny(), N=0)) == 0


def test_admission_fifo_budget_and_slots(L):
    # fits two, third blocks the rest even though the fourth would fit
    k, adm = L.admission_plan([10, 20, 30, 5], 0, 40, 0, 8)
    assert (k, adm) == (2, [1, 1, 0, 0])
    # slots
    k, adm = L.admission_plan([1, 1, 1], 0, 0, 62, 64)
    assert (k, adm) == (2, [1, 1, 0])
    # a job larger than the whole budget can never run and does not block others
    k, adm = L.admission_plan([50, 10], 0, 40, 0, 8)
    assert (k, adm) == (1, [-1, 1])
    # bytes already in use count against the budget
    k, adm = L.admission_plan([15], 30, 40, 1, 8)
    assert (k, adm) == (0, [0])
    # no budget: only slots limit
    k, adm = L.admission_plan([10**12] * 3, 0, 0, 0, 2)
    assert (k, adm) == (2, [1, 1, 0])


def test_stft_frame_count(L):
    """nfhmm_stft_frames: T = 1 + (n - nfft) // hop, 0 without a whole frame."""
    assert L.stft_frames(1024, 256, 256_768) == 1000
    assert L.stft_frames(1024, 256, 1024) == 1
    assert L.stft_frames(1024, 256, 1023) == 0
    assert L.stft_frames(2048, 512, 2048 + 3 * 512 + 511) == 4


def test_istft_binding_checks_shapes_before_the_call(L):
    """The host inverse takes mag [T][F], [S][T][F] or [B][S][T][F] with phase
    [T][F] or [B][T][F]; a phase of another shape is refused before anything
    reaches the library (no context is needed to see it)."""
    with pytest.raises(ValueError):
        L.istft(None, np.zeros((2, 3, 10, 33), np.float32), np.zeros((3, 10, 33), np.float32), 300, 64, 16)
    with pytest.raises(ValueError):
        L.istft(None, np.zeros((2, 10, 33), np.float32), np.zeros((10, 32), np.float32), 300, 64, 16)
    with pytest.raises(ValueError):   # several mixtures need one phase each
        L.istft(None, np.zeros((2, 3, 10, 33), np.float32), np.zeros((10, 33), np.float32), 300, 64, 16)
