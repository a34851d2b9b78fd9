"""GPU parity of the split-BF16 precision form against the FP64 oracle.

The split-BF16 form evaluates the same-level (batched) M2L as BF16
matrix-core products (FP32 accumulation), every other operator in FP32.
Representing an FP32 value as a sum of two BF16 values keeps 16 significand
bits: the low multipole degrees (coefficient index k < 32) take hi*hi + hi*lo +
lo*hi (relative error of order 2^-16 per product), the higher degrees, whose
share of the result decays like the expansion's terms, take hi*hi + hi*lo
(k < 48, 2^-9) or hi*hi alone (2^-8); the bar stays the one of the
FP32 form: potential within 1e-5 and field within 1e-4 relative L2 of the
oracle's FMM on the same lists at p = 10, and of the FP64 direct sum at the
full 4,194,304-particle Plummer size on seeded targets; at p = 12 (storage
width 192) the same bar holds against the oracle's FMM and against the direct
sum on 2,000 seeded targets of the full 16,777,216-particle Plummer set.
"""
import numpy as np
import pytest

import oracle as ora
import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

BF16 = 1


def as_f32(a):
    return np.asarray(a, dtype=np.float32).astype(np.float64)


def run(x, y, z, q, p, theta, ncrit, precision, policy=0, f=None):
    from paper_1108_5815_amd import FMM
    f = f or FMM(0)
    f.build_tree(*(torch.tensor(a, dtype=torch.float32, device="cuda:0") for a in (x, y, z, q)), ncrit)
    f.traverse(p, theta, policy)
    phi, E = f.evaluate(precision, out_dtype=torch.float64)
    torch.cuda.synchronize()
    return f, phi.cpu().numpy(), E.cpu().numpy().T


@pytest.mark.parametrize("p", [4, 7, 8, 10, 12])
def test_bf16_uniform_vs_oracle(p):
    """Each supported padded width (32, 64, 96, 128, 192 coefficients)."""
    n = 24000
    x, y, z = (as_f32(a) for a in synth.uniform_cube(n, 21))
    q = as_f32(synth.charges_uniform(n, 121))
    f, phi, E = run(x, y, z, q, p, 0.5, 48, BF16)
    assert f.m2l_split()[0] > 0          # the batched path ran
    po, Eo, _ = ora.fmm(x, y, z, q, p, 0.5, 48)
    ep, eE = ora.rel_l2(phi, po), ora.rel_l2(E, Eo)
    print(f"p={p}: split-bf16 vs oracle FMM phi {ep:.2e} E {eE:.2e}")
    assert ep < 1e-5 and eE < 1e-4


@pytest.mark.parametrize("theta", [0.5, 0.4])
def test_bf16_plummer_adaptive(theta):
    n = 20000
    x, y, z = (as_f32(a) for a in synth.plummer(n, 22))
    q = as_f32(synth.charges_equal(n))
    f, phi, E = run(x, y, z, q, 10, theta, 16, BF16)
    po, Eo, _ = ora.fmm(x, y, z, q, 10, theta, 16)
    assert ora.rel_l2(phi, po) < 1e-5 and ora.rel_l2(E, Eo) < 1e-4


def test_bf16_close_to_fp32_locals():
    """Same lists, two precisions: locals differ by the BF16 split's rounding only."""
    n = 30000
    x, y, z = (as_f32(a) for a in synth.uniform_cube(n, 23))
    q = as_f32(synth.charges_uniform(n, 123))
    f, phi32, _ = run(x, y, z, q, 10, 0.5, 32, 0)
    _, L32 = f.expansions()
    phi16 = f.evaluate(BF16, out_dtype=torch.float64)[0].cpu().numpy()
    _, L16 = f.expansions()
    d = np.abs(L16 - L32).max() / np.abs(L32).max()
    assert 0 < d < 2e-5
    assert ora.rel_l2(phi16, phi32) < 5e-6


def test_bf16_deterministic():
    x, y, z = synth.plummer(20000, 24)
    q = synth.charges_uniform(20000, 124)
    _, a, Ea = run(x, y, z, q, 10, 0.4, 32, BF16)
    _, b, Eb = run(x, y, z, q, 10, 0.4, 32, BF16)
    assert np.array_equal(a, b) and np.array_equal(Ea, Eb)


def test_bf16_unsupported_orders():
    from paper_1108_5815_amd import FMM, FMMError
    f = FMM(0)
    x = torch.rand(2000, device="cuda:0")
    f.build_tree(x, x.flip(0), x * 0.5, x, 16)
    for p in (13, 16):
        f.traverse(p, 0.5, 0)
        with pytest.raises(FMMError) as e:
            f.evaluate(BF16)
        assert e.value.status == 5
        f.evaluate(0)                    # FP32 still works on the same lists
    with pytest.raises(FMMError) as e:
        f.evaluate(2)                    # no such precision form
    assert e.value.status == 1


def test_full_size_plummer4m_p10_bf16_sampled():
    """4,194,304 Plummer points, FP32 inputs, p = 10, theta = 0.4, ncrit = 64,
    split-BF16 M2L: 1,000 seeded targets against the FP64 direct sum."""
    x, y, z, q, tg, w = synth.make_workload("plummer4m_p10")
    xs, ys, zs, qs = (as_f32(a) for a in (x, y, z, q))
    f, phi, E = run(xs, ys, zs, qs, w["p"], w["theta"], w["ncrit"], BF16)
    pd, Ed = ora.direct(xs, ys, zs, qs, tg)
    ep, eE = ora.rel_l2(phi[tg], pd), ora.rel_l2(E[tg], Ed)
    print(f"plummer4m p10 split-bf16: phi rel L2 {ep:.3e}  E rel L2 {eE:.3e}")
    assert ep < 1e-5 and eE < 1e-4


def test_full_size_plummer16m_p12_bf16_sampled():
    """16,777,216 Plummer points, FP32 inputs, p = 12, theta = 0.4, ncrit = 64,
    split-BF16 M2L (the widest storage, 192 coefficients): 2,000 seeded targets
    against the FP64 direct sum."""
    x, y, z, q, tg, w = synth.make_workload("plummer16m_p12")
    xs, ys, zs, qs = (as_f32(a) for a in (x, y, z, q))
    f, phi, E = run(xs, ys, zs, qs, w["p"], w["theta"], w["ncrit"], BF16)
    assert f.m2l_split()[0] > 0
    pd, Ed = ora.direct(xs, ys, zs, qs, tg)
    ep, eE = ora.rel_l2(phi[tg], pd), ora.rel_l2(E[tg], Ed)
    print(f"plummer16m p12 split-bf16: phi rel L2 {ep:.3e}  E rel L2 {eE:.3e}")
    assert ep < 1e-5 and eE < 1e-4
