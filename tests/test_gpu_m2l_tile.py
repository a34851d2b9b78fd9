"""Tile width of the same-level M2L GEMM (fmm_set_m2l_tile): at storage width
128 (p = 10) tiles of 64 and of 128 targets give identical values in both
precisions (a row's products and their order do not depend on which other
rows share its tile: slots a row does not use read the all-zero row), agree
with the oracle's FMM, and the autotuner keeps one of the two."""
import numpy as np
import pytest

import oracle as ora
import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _f32(a):
    return np.asarray(a, np.float32).astype(np.float64)


def _dev(a):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float32, device="cuda:0")


@pytest.mark.parametrize("precision", [0, 1], ids=["fp32", "split_bf16"])
def test_tile_widths_identical(precision):
    from paper_1108_5815_amd import FMM
    n = 60000
    x, y, z = (_f32(a) for a in synth.plummer(n, 41))
    q = _f32(synth.charges_uniform(n, 42))
    f = FMM(0)
    t = [_dev(a) for a in (x, y, z, q)]
    out = {}
    for cols in (64, 128):
        f.set_m2l_tile(cols)
        f.build_tree(*t, 64)
        f.traverse(10, 0.5, 0)
        assert f.m2l_tile() == cols
        shape = f.gemm_shape()
        phi, E = f.evaluate(precision, out_dtype=torch.float64)
        torch.cuda.synchronize()
        out[cols] = (phi.cpu().numpy(), E.cpu().numpy(), shape)
    print("gemm shapes", out[64][2], out[128][2])
    assert out[128][2]["tiles"] < out[64][2]["tiles"]
    assert np.array_equal(out[64][0], out[128][0]) and np.array_equal(out[64][1], out[128][1])
    po, Eo, _ = ora.fmm(x, y, z, q, 10, 0.5, 64)
    tol = 1e-5 if precision == 0 else 2e-5
    assert ora.rel_l2(out[128][0], po) < tol and ora.rel_l2(out[128][1].T, Eo) < 10 * tol


def test_autotune_picks_a_width():
    from paper_1108_5815_amd import FMM
    n = 200000
    x, y, z = (_f32(a) for a in synth.plummer(n, 43))
    q = _f32(synth.charges_uniform(n, 44))
    f = FMM(0)
    f.build_tree(*[_dev(a) for a in (x, y, z, q)], 64)
    f.traverse(10, 0.4, 0)
    phi0, _ = f.evaluate(1, out_dtype=torch.float64)
    cfg = f.autotune(1, reps=2)
    assert cfg["m2l_tile"] in (64, 128) and f.m2l_tile() == cfg["m2l_tile"]
    phi1, _ = f.evaluate(1, out_dtype=torch.float64)
    torch.cuda.synchronize()
    print("autotune", cfg)
    assert ora.rel_l2(phi1.cpu().numpy(), phi0.cpu().numpy()) < 1e-6
    with pytest.raises(Exception):
        f.set_m2l_tile(96)
