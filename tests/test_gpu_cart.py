"""The Cartesian (Taylor) expansion family on the GPU against the oracle's
Cartesian method on the same lists: expansions coefficient by coefficient,
values under the three policies and both precisions, pairs beyond the class
key, targets that differ from the sources, and the order-based switch of
FMM_EXPANSION_AUTO ("Hybrid treecode/FMM algorithm": switch to Cartesian
expansions when the required accuracy is low)."""
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


def run_cart(x, y, z, q, p, theta, ncrit, policy=0, costs=None, precision=0):
    from paper_1108_5815_amd import EXPANSION_CARTESIAN, FMM
    f = FMM(0)
    f.set_expansion(EXPANSION_CARTESIAN)
    f.build_tree(_dev(x), _dev(y), _dev(z), _dev(q), ncrit)
    if costs is not None:
        f.set_costs(*costs)
    f.traverse(p, theta, policy)
    assert f.expansion() == EXPANSION_CARTESIAN
    phi, E = f.evaluate(precision, out_dtype=torch.float64)
    torch.cuda.synchronize()
    return f, phi.cpu().numpy(), E.cpu().numpy().T


def oracle_cart(x, y, z, q, p, theta, ncrit, policy=0, costs=(0, 0, 0)):
    t = ora.Tree(x, y, z, ncrit)
    t.traverse(theta, policy, costs)
    phi, E = t.evaluate_cart(p, q)
    return t, phi, E


def _degrees(p):
    return np.array([n for n in range(p + 1) for a in range(n, -1, -1) for b in range(n - a, -1, -1)])


def test_cartesian_expansions_match_oracle():
    n, p = 8000, 4
    x, y, z = (_f32(a) for a in synth.plummer(n, 91))
    q = _f32(synth.charges_uniform(n, 191))
    f, _, _ = run_cart(x, y, z, q, p, 0.5, 20)
    Mg, Lg = f.expansions()
    t, _, _ = oracle_cart(x, y, z, q, p, 0.5, 20)
    Mo, Lo = t.expansions_cart()
    r = t.cells()["radius"][:, None]
    deg = _degrees(p)[None, :]
    Mref = Mo / r ** deg
    Lref = Lo * r ** (deg + 1)
    assert Mg.shape == Mref.shape
    assert np.abs(Mg - Mref).max() <= 1e-5 * np.abs(Mref).max()
    assert np.abs(Lg - Lref).max() <= 1e-5 * np.abs(Lref).max()


@pytest.mark.parametrize("p", [2, 4, 6])
@pytest.mark.parametrize("policy,costs", [(0, None), (1, None), (2, (40.0, 2.0, 1.0))],
                         ids=["fmm", "treecode", "hybrid"])
def test_cartesian_values_match_oracle(p, policy, costs):
    n = 12000
    x, y, z = (_f32(a) for a in synth.plummer(n, 92))
    q = _f32(synth.charges_uniform(n, 192))
    for theta in (0.5, 0.4):
        _, phi, E = run_cart(x, y, z, q, p, theta, 24, policy, costs)
        _, po, Eo = oracle_cart(x, y, z, q, p, theta, 24, policy, costs or (0, 0, 0))
        assert ora.rel_l2(phi, po) < 1e-5 and ora.rel_l2(E, Eo) < 1e-4, (p, theta)


@pytest.mark.parametrize("p", [3, 4, 6])
def test_cartesian_split_bf16(p):
    n = 16000
    x, y, z = (_f32(a) for a in synth.uniform_cube(n, 93))
    q = _f32(synth.charges_uniform(n, 193))
    f, phi, E = run_cart(x, y, z, q, p, 0.5, 32, precision=1)
    assert f.m2l_split()[0] > 0
    _, po, Eo = oracle_cart(x, y, z, q, p, 0.5, 32)
    assert ora.rel_l2(phi, po) < 1e-5 and ora.rel_l2(E, Eo) < 1e-4


def test_cartesian_pairs_beyond_the_class_key():
    from test_gpu_parity import deep_pair_set
    x, y, z = (_f32(a) for a in deep_pair_set())
    q = _f32(synth.charges_uniform(x.size, 194))
    _, phi, E = run_cart(x, y, z, q, 5, 0.5, 64)
    t, po, Eo = oracle_cart(x, y, z, q, 5, 0.5, 64)
    c = t.cells()
    a, b = t.lists()[0]
    assert (np.abs(c["level"][a] - c["level"][b]) > 8).sum() > 50
    assert ora.rel_l2(phi, po) < 1e-5 and ora.rel_l2(E, Eo) < 1e-4


def test_cartesian_targets_sources():
    from paper_1108_5815_amd import EXPANSION_CARTESIAN, FMM
    tg = _f32(np.stack(synth.uniform_cube(3000, 95), 1) * 2.4 - 1.2)
    sr = _f32(np.stack(synth.sphere_shell(5000, 96), 1))
    q = _f32(synth.charges_uniform(5000, 97))
    f = FMM(0)
    f.set_expansion(EXPANSION_CARTESIAN)
    f.build_tree_ts([_dev(tg[:, d]) for d in range(3)], [_dev(sr[:, d]) for d in range(3)], _dev(q), 24)
    f.traverse(5, 0.5, 0)
    phi, E = f.evaluate(out_dtype=torch.float64)
    t = ora.Tree.targets_sources(tg, sr, 24)
    t.traverse(0.5, 0)
    po, Eo = t.evaluate_cart(5, q)
    assert ora.rel_l2(phi.cpu().numpy(), po) < 1e-5 and ora.rel_l2(E.cpu().numpy().T, Eo) < 1e-4


def test_auto_switch_by_order():
    from paper_1108_5815_amd import EXPANSION_AUTO, EXPANSION_CARTESIAN, EXPANSION_SPHERICAL, FMM, FMMError
    n = 6000
    x, y, z = (_f32(a) for a in synth.plummer(n, 98))
    q = _f32(synth.charges_uniform(n, 198))
    f = FMM(0)
    f.build_tree(_dev(x), _dev(y), _dev(z), _dev(q), 24)
    f.set_expansion(EXPANSION_AUTO, 3)
    pd, Ed = ora.direct(x, y, z, q)
    for p, fam in ((2, EXPANSION_CARTESIAN), (3, EXPANSION_CARTESIAN), (4, EXPANSION_SPHERICAL),
                   (10, EXPANSION_SPHERICAL)):
        f.traverse(p, 0.5, 0)
        assert f.expansion() == fam
        phi, E = f.evaluate(out_dtype=torch.float64)
        e = ora.rel_l2(phi.cpu().numpy(), pd)
        print("auto p", p, "family", fam, "phi error vs direct", e)
    f.set_expansion(EXPANSION_CARTESIAN)
    with pytest.raises(FMMError) as err:
        f.traverse(7, 0.5, 0)
    assert err.value.status == 5
    with pytest.raises(FMMError):
        f.set_expansion(EXPANSION_AUTO, 9)
