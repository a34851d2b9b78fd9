"""The kernels of the M2L pairs outside the same-level GEMM: class-batched
matrix-core products, dense per-pair, and rotation-based per-pair (rotate the
multipole to the offset's axis, translate along it, rotate back; "Dual tree
traversal" names rotation-based translation as one of the per-pair
choices).  Each against the oracle's FMM on the same lists."""
import numpy as np
import pytest

import oracle as ora
import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

KINDS = [0, 1, 2, 3]
NAMES = ["class_dense", "class_rotation", "pair_dense", "pair_rotation"]


def _f32(a):
    return np.asarray(a, np.float32).astype(np.float64)


def _dev(a):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float32, device="cuda:0")


def run(x, y, z, q, p, theta, ncrit, kind):
    from paper_1108_5815_amd import FMM
    f = FMM(0)
    f.set_m2l_kernel(kind)
    f.build_tree(_dev(x), _dev(y), _dev(z), _dev(q), ncrit)
    f.traverse(p, theta, 0)
    phi, E = f.evaluate(out_dtype=torch.float64)
    torch.cuda.synchronize()
    return f, phi.cpu().numpy(), E.cpu().numpy().T


@pytest.mark.parametrize("kind", KINDS, ids=NAMES)
@pytest.mark.parametrize("p", [4, 10, 16])
def test_m2l_kinds_match_oracle(kind, p):
    n = 9000
    x, y, z = (_f32(a) for a in synth.plummer(n, 71))
    q = _f32(synth.charges_uniform(n, 171))
    for theta in (0.5, 0.4):
        f, phi, E = run(x, y, z, q, p, theta, 16, kind)
        assert f.m2l_split()[1] > 0            # there are pairs outside the GEMM
        po, Eo, _ = ora.fmm(x, y, z, q, p, theta, 16)
        assert ora.rel_l2(phi, po) < 1e-5 and ora.rel_l2(E, Eo) < 1e-4, (p, theta)


@pytest.mark.parametrize("kind", [1, 3], ids=["class_rotation", "pair_rotation"])
def test_rotation_beyond_the_class_key(kind):
    from test_gpu_parity import deep_pair_set
    x, y, z = (_f32(a) for a in deep_pair_set())
    q = _f32(synth.charges_uniform(x.size, 172))
    _, phi, E = run(x, y, z, q, 12, 0.5, 64, kind)
    po, Eo, _ = ora.fmm(x, y, z, q, 12, 0.5, 64)
    assert ora.rel_l2(phi, po) < 1e-5 and ora.rel_l2(E, Eo) < 1e-4


def test_autotune_picks_a_kind_and_keeps_values():
    from paper_1108_5815_amd import FMM
    n = 60000
    x, y, z = (_f32(a) for a in synth.plummer(n, 73))
    q = _f32(synth.charges_uniform(n, 173))
    f = FMM(0)
    f.build_tree(_dev(x), _dev(y), _dev(z), _dev(q), 32)
    f.traverse(12, 0.4, 0)
    ref, Eref = f.evaluate(out_dtype=torch.float64)
    cfg = f.autotune(0, reps=2)
    assert cfg["m2l_kernel"] in KINDS
    got, Egot = f.evaluate(out_dtype=torch.float64)
    torch.cuda.synchronize()
    print("autotuned", cfg)
    assert ora.rel_l2(got.cpu().numpy(), ref.cpu().numpy()) < 1e-6
