"""Host-side checks of the C ABI (no GPU needed): the library loads, exports
every entry point include/lsr.h declares, and the pure host entry points
(defaults, workspace sizing, argument validation) behave as documented."""
import math
import os
import re

import pytest

from paper_2410_22205_amd import lsr

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    text = open(os.path.join(ROOT, "include", "lsr.h")).read()
    return sorted(set(re.findall(r"\b(lsr_[a-z_]+)\s*\(", text)))


def test_header_and_binding_agree():
    assert sorted(lsr.EXPORTED) == _declared()


def test_library_exports_every_declared_symbol():
    lib = lsr.load()
    for name in _declared():
        assert hasattr(lib, name), name


def test_params_default_follow_the_paper():
    for dim, g, b in [(2, 4, 2), (3, 6, 3)]:
        p = lsr.lsr_params_default(dim, 0.1)
        assert p.gamma == pytest.approx(g * 0.1) and p.beta == pytest.approx(b * 0.1)
        assert p.grad_C == 1e-3 and p.grad_alpha == 1.0 and p.p == 1.0 and p.delta == 1.0
        assert p.reinit_dtau == pytest.approx(0.05)
        assert p.reinit_iters == math.ceil((p.gamma + 0.1) / 0.05 - 1e-9)


def test_workspace_bytes_scale_with_grid_and_cloud():
    g = lsr.make_grid({"dim": 3, "n": (64, 64, 64), "lo": (-1, -1, -1), "h": 2 / 63})
    a = lsr.lsr_workspace_bytes(g, None, 1000)
    b = lsr.lsr_workspace_bytes(g, None, 100000)
    assert b > a > 64 ** 3 * 40
    g2 = lsr.make_grid({"dim": 3, "n": (128, 64, 64), "lo": (-1, -1, -1), "h": 2 / 63})
    assert lsr.lsr_workspace_bytes(g2, None, 1000) > 1.9 * a
    p64 = lsr.lsr_params_default(3, 2 / 63)
    p64.precision = lsr.LSR_FP64
    assert lsr.lsr_workspace_bytes(g, p64, 1000) > a + 64 ** 3 * 20


@pytest.mark.parametrize("grid,code", [
    ({"dim": 4, "n": (8, 8, 8), "lo": (0, 0, 0), "h": 0.1}, lsr.LSR_E_INVALID),
    ({"dim": 3, "n": (3, 8, 8), "lo": (0, 0, 0), "h": 0.1}, lsr.LSR_E_INVALID),
    ({"dim": 3, "n": (8, 8, 8), "lo": (0, 0, 0), "h": 0.0}, lsr.LSR_E_INVALID),
    ({"dim": 3, "n": (8, 8, 8), "lo": (float("nan"), 0, 0), "h": 0.1}, lsr.LSR_E_INVALID),
    ({"dim": 3, "n": (4096, 4096, 300), "lo": (0, 0, 0), "h": 0.1}, lsr.LSR_E_UNSUPPORTED),
])
def test_invalid_grids_are_rejected(grid, code):
    with pytest.raises(lsr.LsrError) as e:
        lsr.lsr_workspace_bytes(lsr.make_grid(grid), None, 10)
    assert e.value.status == code
    assert lsr.lsr_last_error()


def _create(params_over):
    g = lsr.make_grid({"dim": 3, "n": (8, 8, 8), "lo": (0, 0, 0), "h": 0.1})
    p = lsr.lsr_params_default(3, 0.1)
    for k, v in params_over.items():
        setattr(p, k, v)
    # validation happens before any device call, so a dummy pointer is safe
    return lsr.lsr_create(g, p, 256, 1 << 30, 0)


@pytest.mark.parametrize("over,code", [
    ({"beta": 0.7}, lsr.LSR_E_INVALID),          # beta >= gamma
    ({"delta": -1.0}, lsr.LSR_E_INVALID),
    ({"p": 3.0}, lsr.LSR_E_UNSUPPORTED),         # the paper runs p = 1 and 2
    ({"p": 0.5}, lsr.LSR_E_INVALID),
    ({"reinit_dtau": 0.1}, lsr.LSR_E_INVALID),   # beyond h/sqrt(3)
    ({"reinit_every": -1}, lsr.LSR_E_INVALID),
    ({"precision": 7}, lsr.LSR_E_INVALID),
])
def test_invalid_params_are_rejected(over, code):
    with pytest.raises(lsr.LsrError) as e:
        _create(over)
    assert e.value.status == code


def test_misaligned_or_small_workspace_is_rejected():
    g = lsr.make_grid({"dim": 3, "n": (8, 8, 8), "lo": (0, 0, 0), "h": 0.1})
    p = lsr.lsr_params_default(3, 0.1)
    with pytest.raises(lsr.LsrError) as e:
        lsr.lsr_create(g, p, 256 + 4, 1 << 30, 0)
    assert e.value.status == lsr.LSR_E_INVALID
    with pytest.raises(lsr.LsrError) as e:
        lsr.lsr_create(g, p, 256, 1024, 0)
    assert e.value.status == lsr.LSR_E_NOMEM


def test_tune_cache_file_is_checked(tmp_path):
    good = tmp_path / "tune.txt"
    good.write_text("# dim fp64 q1 weno nodes lanes bpc ms\n3 0 1 1 1048576 4 2 0.5\n")
    lsr.lsr_set_tune_cache(str(good))
    bad = tmp_path / "bad.txt"
    bad.write_text("3 0 1 1 1048576 four 2 0.5\n")
    with pytest.raises(lsr.LsrError) as e:
        lsr.lsr_set_tune_cache(str(bad))
    assert e.value.status == lsr.LSR_E_INVALID
    lsr.lsr_set_tune_cache(str(tmp_path / "missing.txt"))  # an empty cache
    lsr.lsr_set_tune_cache(None)
