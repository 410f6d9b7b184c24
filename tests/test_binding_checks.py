"""The Python binding refuses wrong tensors before any library call: element
type against the grid's precision (FP64 sides of hj_solve_mixed and
hj_tube_finish), node count (times the output count for hj_solve_outputs),
contiguity and device.  CPU only: a CPU tensor must never reach a kernel."""
import pytest

torch = pytest.importorskip("torch")


def _grid(prec, n=(5, 4, 3)):
    from paper_2507_11542_amd import hj

    g = object.__new__(hj.Grid)  # no device: only the checks are exercised
    g.n, g.prec, g.handle = n, prec, None
    return g


def test_check_array_rejects():
    from paper_2507_11542_amd.hj import _check_array

    ok_cpu = torch.zeros(60, dtype=torch.float64)
    with pytest.raises(ValueError, match="dtype"):
        _check_array(torch.zeros(60, dtype=torch.float32), "float64", 60, "V")
    with pytest.raises(ValueError, match="elements"):
        _check_array(torch.zeros(59, dtype=torch.float64), "float64", 60, "V")
    with pytest.raises(ValueError, match="contiguous"):
        _check_array(torch.zeros(120, dtype=torch.float64)[::2], "float64", 60, "V")
    with pytest.raises(ValueError, match="GPU"):
        _check_array(ok_cpu, "float64", 60, "V")
    _check_array(None, "float64", 60, "V")      # optional arrays
    _check_array(12345, "float64", 60, "V")     # raw device pointers pass through


def test_grid_methods_check_before_calling():
    g64, g32 = _grid("fp64"), _grid("fp32")
    f64 = torch.zeros(g64.points, dtype=torch.float64)
    f32 = torch.zeros(g32.points, dtype=torch.float32)
    with pytest.raises(ValueError, match="V0: dtype"):
        g64.solve(f32, f64, 0.0, 1.0)
    with pytest.raises(ValueError, match="GPU"):
        g64.solve(f64, f64, 0.0, 1.0)
    with pytest.raises(ValueError, match="V_outs: 60 elements, expected 120"):
        g64.solve_outputs(None, f64, 0.0, [0.5, 1.0])
    with pytest.raises(ValueError, match="V0: dtype"):
        g32.solve_mixed(f32, f64, 0.0, 1.0)
    with pytest.raises(ValueError, match="V32: dtype"):
        g32.tube_finish(f64, f64, f64)
    with pytest.raises(ValueError, match="V: dtype"):
        g32.step(f64, None, 0.0, 1.0)
    with pytest.raises(ValueError, match="L_out"):
        g32.rhs(None, torch.zeros(7, dtype=torch.float32))


def test_batch_checks_every_instance():
    from paper_2507_11542_amd import hj

    grids = [_grid("fp32"), _grid("fp32", (3, 3, 3))]
    v0s = [None, None]
    outs = [None, torch.zeros(26, dtype=torch.float32)]
    with pytest.raises(ValueError, match=r"Vouts\[1\]: 26 elements"):
        hj.Batch._check(grids, (v0s, "V0s"), (outs, "Vouts"))
    with pytest.raises(ValueError, match="1 arrays for 2 grids"):
        hj.Batch._check(grids, ([None], "V0s"))
