"""C-ABI checks that need no GPU: the library loads, exports every entry point
include/umbir.h declares, and rejects invalid input before any HIP call."""
import ctypes as C
import os
import re

import pytest

from synth import card_c1, card_c2, card_c3, tiny_card
from synth.cards import Prior

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
umbir = pytest.importorskip("paper_2202_09703_amd.umbir",
                            reason="libumbir.so not built (python -m paper_2202_09703_amd.build)")


def _declared():
    text = open(os.path.join(ROOT, "include", "umbir.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(umbir_[a-z_]+)\s*\(", text)))


def test_exports_every_declared_symbol():
    lib = C.CDLL(umbir.library_path())
    names = _declared()
    assert len(names) >= 10
    for n in names:
        assert hasattr(lib, n), f"{n} declared in umbir.h but not exported"
    assert sorted(umbir.EXPORTS) == names


def test_strerror():
    for st in (0, -1, -2, -3, -4, -5):
        assert umbir._lib.umbir_strerror(st).decode()
    assert umbir._lib.umbir_strerror(99).decode() == "unknown status"


def _build_status(card):
    pb = umbir.Problem(card)
    h = C.c_void_p()
    st = umbir._lib.umbir_build_geometry(C.byref(pb.c), None, C.byref(h))
    return st, umbir._lib.umbir_last_error().decode()


def _with(card, **changes):
    import dataclasses
    parts = {}
    for field, val in changes.items():
        part, attr = field.split("__")
        parts.setdefault(part, {})[attr] = val
    kw = {p: dataclasses.replace(getattr(card, p), **v) for p, v in parts.items()}
    return dataclasses.replace(card, **kw)


@pytest.mark.parametrize("changes,status", [
    ({"medium__speed": (1480.0, -5900.0, 3000.0)}, umbir.EINVAL),
    ({"medium__thickness": (10e-3, 0.0)}, umbir.EINVAL),
    ({"medium__density": (1000.0, 7850.0, float("nan"))}, umbir.EINVAL),
    ({"medium__atten": (0.0, -2e-6, 0.0)}, umbir.EINVAL),
    ({"medium__atten": (0.0, 2e-6, 0.0), "acq__storage": 1}, umbir.ENOTSUP),  # attenuation needs FP32
    ({"medium__atten": (0.0, 2e-6, 0.0), "acq__n_gamma": 1}, umbir.EINVAL),
    ({"medium__atten": (0.0, 2e-6, 0.0), "acq__n_gamma": 65}, umbir.EINVAL),
    ({"grid__nx": 0}, umbir.EINVAL),
    ({"grid__dz": -1e-3}, umbir.EINVAL),
    ({"array__beta": -1}, umbir.EINVAL),
    ({"array__tx_x": (0.1e-3,)}, umbir.ENOTSUP),
    ({"array__rx_offset": (0.0, 1.1e-3)}, umbir.ENOTSUP),
    ({"acq__t_win": 12.05e-6}, umbir.EINVAL),
    ({"acq__oversample": 48}, umbir.ENOTSUP),
    ({"acq__oversample": 0}, umbir.ENOTSUP),
    ({"acq__fs": 0.0}, umbir.EINVAL),
    ({"acq__storage": 3}, umbir.EINVAL),
    ({"acq__storage": -1}, umbir.EINVAL),
    ({"acq__storage": 1, "acq__oversample": 16}, umbir.ENOTSUP),  # 16-bit needs Q = 32 or 64
    ({"acq__storage": 2, "acq__oversample": 8}, umbir.ENOTSUP),
])
def test_invalid_problems_rejected_without_device(changes, status):
    st, msg = _build_status(_with(card_c1(), **changes))
    assert st == status, msg
    assert msg


def test_layer_count_limits():
    import dataclasses
    card = card_c1()
    med = dataclasses.replace(card.medium, speed=(), thickness=(), atten=(), density=())
    assert _build_status(dataclasses.replace(card, medium=med))[0] == umbir.EINVAL


def test_estimate_bytes():
    assert umbir.estimate_bytes(card_c1()) > 0
    b2, b3 = umbir.estimate_bytes(card_c2()), umbir.estimate_bytes(card_c3())
    assert 0 < b2 < b3
    assert umbir.estimate_bytes(_with(card_c1(), grid__nx=-3)) == 0


@pytest.mark.parametrize("kw,ok", [
    ({}, True), ({"p": 2.0}, True), ({"p": 1.0}, False), ({"q": 1.8}, False), ({"p": 2.2, "q": 2.0}, False),
    ({"T": 0.0}, False), ({"sigma0": -1.0}, False), ({"m": 0.0}, False), ({"a": -0.5}, False),
])
def test_prior_checked_before_any_device_call(kw, ok):
    """umbir_reconstruct validates the prior before touching the geometry or
    the device, so placeholder pointers are never dereferenced here."""
    import dataclasses
    pr = umbir.make_prior(dataclasses.replace(Prior(), **kw), 0.01)
    if ok:
        return  # a valid prior would go on to use the device
    fake = C.c_void_p(16)
    st = umbir._lib.umbir_reconstruct(fake, C.byref(pr), fake, 3, fake, fake, None, None, 0, None)
    assert st == umbir.EINVAL
    bad_sigma = umbir.make_prior(Prior(), 0.0)
    assert umbir._lib.umbir_reconstruct(fake, C.byref(bad_sigma), fake, 3, fake, fake, None, None, 0,
                                        None) == umbir.EINVAL


def test_null_arguments():
    lib = umbir._lib
    assert lib.umbir_forward(None, None, None, 0, None, 0, None) == umbir.EINVAL
    assert lib.umbir_adjoint(None, None, None, None, 0, None) == umbir.EINVAL
    assert lib.umbir_direct(None, None, None, 0, None) == umbir.EINVAL
    assert lib.umbir_build_geometry(None, None, None) == umbir.EINVAL
    lib.umbir_geometry_free(None)
    assert lib.umbir_geometry_bytes(None) == 0
    assert lib.umbir_workspace_bytes(None, 0) == 0


def test_solver_arguments_checked_before_any_device_call():
    lib = umbir._lib
    fake = C.c_void_p(16)
    out = C.c_void_p()
    pr = umbir.make_prior(Prior(), 0.01)
    assert lib.umbir_solver_create(None, C.byref(pr), fake, None, None, 5, None, C.byref(out)) == umbir.EINVAL
    assert lib.umbir_solver_create(fake, C.byref(pr), None, None, None, 5, None, C.byref(out)) == umbir.EINVAL
    assert lib.umbir_solver_create(fake, C.byref(pr), fake, None, None, -1, None, C.byref(out)) == umbir.EINVAL
    bad = umbir.make_prior(Prior(p=0.9), 0.01)
    assert lib.umbir_solver_create(fake, C.byref(bad), fake, None, None, 5, None, C.byref(out)) == umbir.EINVAL
    assert lib.umbir_solver_step(None, 1, None) == umbir.EINVAL
    assert lib.umbir_solver_read(None, None, None, None, None) == umbir.EINVAL
    assert lib.umbir_solver_iterations(None) == -1
    assert lib.umbir_solver_bytes(None, 3) == 0
    lib.umbir_solver_free(None)


def test_tuning_and_batch_arguments_checked_before_any_device_call():
    lib = umbir._lib
    t = umbir._Tuning(1024, 4096)
    assert lib.umbir_get_tuning(None, C.byref(t)) == umbir.EINVAL
    assert lib.umbir_set_tuning(None, C.byref(t)) == umbir.EINVAL
    assert lib.umbir_autotune(None, None, C.byref(t)) == umbir.EINVAL
    out = C.c_void_p()
    assert lib.umbir_batch_create(None, 2, 0, C.byref(out)) == umbir.EINVAL
    one = (C.c_void_p * 1)(16)
    assert lib.umbir_batch_create(one, 0, 0, C.byref(out)) == umbir.EINVAL
    assert lib.umbir_batch_create(one, 1, 0, None) == umbir.EINVAL
    assert lib.umbir_batch_create(one, 1, 7, C.byref(out)) == umbir.EINVAL  # unknown mode
    nul = (C.c_void_p * 2)(16, None)
    assert lib.umbir_batch_create(nul, 2, 0, C.byref(out)) == umbir.EINVAL
    dup = (C.c_void_p * 2)(16, 16)
    assert lib.umbir_batch_create(dup, 2, 1, C.byref(out)) == umbir.EINVAL
    assert lib.umbir_batch_step(None, 1, None) == umbir.EINVAL
    lib.umbir_batch_free(None)
