"""The P2P kernel's matrix-core form (tile shapes -1, -2, -4: that many
targets per lane, the sums over sources as FP32 rank-1 updates on
v_mfma_f32_4x4x1f32) against the oracle's direct sum and FMM, and against the
vector form on the same lists.

Cases: every interaction forced to particle-particle sums (the whole
evaluation is then a direct sum through the P2P lists, ancestors' lists
included), leaf sizes from 1 to 64 (ragged blocks of four targets and every
group count), a leaf of more than 64 coincident points (several target
passes and the r = 0 guard), FP64 input (every cell guarded) and targets that
differ from the sources."""
import numpy as np
import pytest

import oracle as ora
import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _f32(a):
    return np.asarray(a, np.float32).astype(np.float64)


def _dev(a, dt=torch.float32):
    return torch.tensor(np.ascontiguousarray(a), dtype=dt, device="cuda:0")


def _run(f, tpl, precision=0):
    f.set_tile_config([tpl] * 4)
    phi, E = f.evaluate(precision, out_dtype=torch.float64)
    torch.cuda.synchronize()
    return phi.cpu().numpy(), E.cpu().numpy().T


def _tree(x, y, z, q, ncrit, dt=torch.float32):
    from paper_1108_5815_amd import FMM
    f = FMM(0)
    f.build_tree(_dev(x, dt), _dev(y, dt), _dev(z, dt), _dev(q, dt), ncrit)
    return f


def test_all_pairs_direct_plummer():
    """Costs that make every accepted pair a particle-particle sum: the
    evaluation is the direct sum, checked on 2,000 sampled targets."""
    n = 30000
    x, y, z = (_f32(a) for a in synth.plummer(n, 61))
    q = _f32(synth.charges_uniform(n, 62))
    f = _tree(x, y, z, q, 64)
    f.set_costs(1.0, 1.0, 1e-9)
    f.traverse(6, 0.5, 2)
    sz = f.sizes()
    assert sz["m2l"] == 0 and sz["m2p"] == 0 and sz["p2p"] > 0, sz
    tg = np.random.default_rng(63).choice(n, 2000, replace=False)
    po, Eo = ora.direct(x, y, z, q, tg)
    errs = {}
    for tpl in (-1, -2, -4, 4):
        phi, E = _run(f, tpl)
        errs[tpl] = (ora.rel_l2(phi[tg], po), ora.rel_l2(E[tg], Eo))
    print("direct sum through P2P lists, rel L2 (phi, E):", errs)
    for tpl, (ep, eE) in errs.items():
        assert ep < 2e-6 and eE < 2e-5, tpl


@pytest.mark.parametrize("shape", [-1, -2, -4])
@pytest.mark.parametrize("ncrit", [1, 3, 13, 27, 64])
def test_leaf_sizes_against_oracle(ncrit, shape):
    n = 4000 if ncrit > 3 else 1500
    x, y, z = (_f32(a) for a in synth.uniform_cube(n, 70 + ncrit))
    q = _f32(synth.charges_uniform(n, 71 + ncrit))
    f = _tree(x, y, z, q, ncrit)
    f.traverse(6, 0.5, 0)
    phi0, E0 = _run(f, shape)
    phi1, E1 = _run(f, 1)
    po, Eo, _ = ora.fmm(x, y, z, q, 6, 0.5, ncrit)
    assert ora.rel_l2(phi0, po) < 1e-5 and ora.rel_l2(E0, Eo) < 1e-4
    assert ora.rel_l2(phi0, phi1) < 2e-6 and ora.rel_l2(E0, E1) < 2e-5


@pytest.mark.parametrize("shape", [-1, -4])
@pytest.mark.parametrize("dt", [torch.float32, torch.float64], ids=["f32", "f64"])
def test_big_coincident_leaf(dt, shape):
    """300 coincident points stop the tree at the level limit: their leaf
    holds more than a wave of targets; coincident pairs contribute nothing."""
    n = 3000
    x, y, z = (_f32(a) for a in synth.uniform_cube(n, 90))
    x[:300], y[:300], z[:300] = 0.3125, 0.5625, 0.4375
    q = _f32(synth.charges_uniform(n, 91))
    f = _tree(x, y, z, q, 32, dt)
    f.set_costs(1.0, 1.0, 1e-9)
    f.traverse(4, 0.5, 2)
    assert f.sizes()["m2l"] == 0
    phi, E = _run(f, shape)
    po, Eo = ora.direct(x, y, z, q)
    assert ora.rel_l2(phi, po) < 2e-6 and ora.rel_l2(E, Eo) < 2e-5
    phi4, E4 = _run(f, 4)
    assert ora.rel_l2(phi, phi4) < 2e-6 and ora.rel_l2(E, E4) < 2e-5


def test_targets_differ_from_sources():
    from paper_1108_5815_amd import FMM
    t = _f32(np.stack(synth.uniform_cube(5000, 95), 1) * 2.4 - 1.2)
    s = _f32(np.stack(synth.sphere_shell(7000, 96), 1))
    q = _f32(synth.charges_uniform(7000, 97))
    f = FMM(0)
    f.build_tree_ts([_dev(t[:, d]) for d in range(3)], [_dev(s[:, d]) for d in range(3)], _dev(q), 20)
    f.traverse(8, 0.5, 0)
    phi, E = _run(f, -2)
    tr = ora.Tree.targets_sources(t, s, 20)
    tr.traverse(0.5, 0)
    po, Eo = tr.evaluate(8, q)
    assert ora.rel_l2(phi, po) < 1e-5 and ora.rel_l2(E, Eo) < 1e-4
    phi4, E4 = _run(f, 4)
    assert ora.rel_l2(phi, phi4) < 2e-6 and ora.rel_l2(E, E4) < 2e-5
