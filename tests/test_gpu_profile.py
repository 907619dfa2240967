"""The library's opt-in kernel timing (umbir_profile_*), through the C ABI:
per-name launch counts and durations, the selection of kernels, the launch
stride used by the benchmark's timed steps, and the reset on collect."""
import pytest

from synth import tiny_card

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
umbir = pytest.importorskip("paper_2202_09703_amd.umbir")


@pytest.fixture(scope="module")
def setup():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    card = tiny_card(n_layers=3, oversample=32)
    geom = umbir.build_geometry(card)
    x = torch.ones(geom.image_shape, dtype=torch.float32, device="cuda:0")
    work = geom.workspace(umbir.WORK_ADJOINT)
    y = umbir.forward(geom, x, work=work)
    torch.cuda.synchronize()
    yield geom, x, y, work
    umbir.profile_enable(False)
    umbir.profile_stride(1)
    umbir.profile_select(None)
    geom.free()


def _pairs(geom, x, y, work, n):
    for _ in range(n):
        umbir.forward(geom, x, y, work=work)
        umbir.adjoint(geom, y, work=work)
    torch.cuda.synchronize()


def test_every_kernel_counted(setup):
    geom, x, y, work = setup
    umbir.profile_select(None)
    umbir.profile_stride(1)
    umbir.profile_enable(True)
    umbir.profile_collect()
    _pairs(geom, x, y, work, 3)
    umbir.profile_enable(False)
    p = umbir.profile_collect()
    for name in ("prescale", "splat", "conv", "corr", "gather"):
        assert name in p, (name, sorted(p))
        assert p[name][1] > 0.0
    assert p["conv"][0] == 3 and p["corr"][0] == 3 and p["splat"][0] == 3
    assert umbir.profile_collect() == {}  # collect resets the totals


def test_selection_and_stride(setup):
    geom, x, y, work = setup
    umbir.profile_enable(True)
    umbir.profile_select(["conv", "corr"])
    umbir.profile_collect()
    _pairs(geom, x, y, work, 7)
    p = umbir.profile_collect()
    assert sorted(p) == ["conv", "corr"] and p["conv"][0] == 7
    umbir.profile_stride(3)  # launches 0, 3, 6 of each selected kernel
    _pairs(geom, x, y, work, 7)
    p = umbir.profile_collect()
    assert p["conv"][0] == 3 and p["corr"][0] == 3
    umbir.profile_stride(1)
    _pairs(geom, x, y, work, 2)
    assert umbir.profile_collect()["conv"][0] == 2
    umbir.profile_enable(False)
    _pairs(geom, x, y, work, 2)
    assert umbir.profile_collect() == {}
    umbir.profile_select(None)
