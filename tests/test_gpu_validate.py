"""fmm_validate on the context's state after builds and traversals of every
kind of input: one set (uniform, clustered, coincident, FP64), targets and
sources apart, a batch forest, and the full-size clustered workload."""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _dev(a, dt=torch.float32):
    return torch.tensor(np.ascontiguousarray(a), dtype=dt, device="cuda:0")


def _check_all_policies(f, p=6, theta=0.5):
    f.set_costs(40.0, 2.0, 1.0)
    for pol in (0, 1, 2):
        f.traverse(p, theta, pol)
        f.validate()


@pytest.mark.parametrize("case", ["uniform", "plummer16", "coincident", "f64"])
def test_one_set(case):
    from paper_1108_5815_amd import FMM
    n = 30000
    if case == "uniform":
        x, y, z = synth.uniform_cube(n, 5)
    else:
        x, y, z = synth.plummer(n, 6)
    x, y, z = (np.array(a) for a in (x, y, z))
    if case == "coincident":
        x[:500], y[:500], z[:500] = 0.1, 0.2, 0.3
    q = synth.charges_uniform(n, 7)
    dt = torch.float64 if case == "f64" else torch.float32
    f = FMM(0)
    f.build_tree(_dev(x, dt), _dev(y, dt), _dev(z, dt), _dev(q, dt), 16 if case == "plummer16" else 64)
    f.validate()
    _check_all_policies(f)


def test_targets_sources_and_batch():
    from paper_1108_5815_amd import FMM
    t = np.stack(synth.uniform_cube(4000, 8), 1) * 2.4 - 1.2
    s = np.stack(synth.sphere_shell(6000, 9), 1)
    q = synth.charges_uniform(6000, 10)
    f = FMM(0)
    f.build_tree_ts([_dev(t[:, d]) for d in range(3)], [_dev(s[:, d]) for d in range(3)], _dev(q), 20)
    f.validate()
    _check_all_policies(f)
    x, y, z, q, off, kinds, tg, w = synth.make_batch("batch256_p8", n_inst=12)
    g = FMM(0)
    g.build_tree_batch(off, _dev(x), _dev(y), _dev(z), _dev(q), 64)
    g.validate()
    _check_all_policies(g, 8)


def test_full_size_plummer4m():
    from paper_1108_5815_amd import FMM
    x, y, z, q, tg, w = synth.make_workload("plummer4m_p10", None)
    f = FMM(0)
    f.build_tree(_dev(x), _dev(y), _dev(z), _dev(q), 64)
    for pol in (0, 1):
        f.traverse(10, 0.4, pol)
        f.validate()
    f.set_m2l_tile(128)
    f.traverse(10, 0.4, 0)
    f.validate()
