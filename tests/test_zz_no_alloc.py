"""fmm_evaluate_noalloc (the evaluation on the library's fixed per-device work
area) against fmm_evaluate, through the C-ABI: the same kernels on the same
tree and lists, so the results must agree bit for bit; two calls in a row, the
second on a smaller input; no allocation inside the call; a clear error beyond
the area's size."""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _tensors(x, y, z, q):
    return [torch.tensor(np.asarray(a, np.float32), device="cuda:0") for a in (x, y, z, q)]


def _outputs(n, dtype):
    return (torch.full((n,), float("nan"), dtype=dtype, device="cuda:0"),
            torch.full((3, n), float("nan"), dtype=dtype, device="cuda:0"))


@pytest.mark.parametrize("precision", [0, 1], ids=["fp32", "split_bf16"])
def test_noalloc_matches_evaluate_twice(precision):
    from paper_1108_5815_amd import FMM
    f = FMM(0)
    ref_ctx = FMM(0)
    cases = [(synth.plummer(40000, 61), synth.charges_uniform(40000, 161), 8, 0.5, 32, torch.float32),
             (synth.uniform_cube(9000, 62), synth.charges_uniform(9000, 162), 10, 0.4, 24, torch.float64)]
    for (x, y, z), q, p, theta, ncrit, od in cases:
        t = _tensors(x, y, z, q)
        n = t[0].numel()
        f.build_tree(*t, ncrit)
        f.traverse(p, theta, 0)
        ref_ctx.build_tree(*t, ncrit)
        ref_ctx.traverse(p, theta, 0)
        ref = ref_ctx.evaluate(precision, out=_outputs(n, od))
        # count the context's allocations while the no-allocation call runs
        calls = []
        f.set_allocator(lambda nb: calls.append(nb) or 0, lambda ptr: None)
        got = f.evaluate_noalloc(precision, out=_outputs(n, od))
        torch.cuda.synchronize()
        f.set_allocator(None, None)
        assert calls == []
        for a, b in zip(got, ref):
            assert torch.equal(a, b), (n, p, theta)
        # and the context's own evaluation on the same lists agrees too
        again = f.evaluate(precision, out=_outputs(n, od))
        for a, b in zip(again, ref):
            assert torch.equal(a, b)


def test_noalloc_rejects_beyond_its_area():
    from paper_1108_5815_amd import FMM, FMMError
    f = FMM(0)
    x, y, z = synth.uniform_cube(1_500_000, 63)
    t = _tensors(x, y, z, synth.charges_uniform(1_500_000, 163))
    f.build_tree(*t, 64)
    f.traverse(10, 0.5, 0)
    with pytest.raises(FMMError) as e:
        f.evaluate_noalloc(0, out=_outputs(1_500_000, torch.float32))
    assert e.value.status == 1 and "bytes of work space" in str(e.value)
    # the context is still usable, and a small problem then fits
    x, y, z = synth.uniform_cube(5000, 64)
    t = _tensors(x, y, z, synth.charges_uniform(5000, 164))
    f.build_tree(*t, 64)
    f.traverse(6, 0.5, 0)
    a = f.evaluate_noalloc(0, out=_outputs(5000, torch.float32))
    b = f.evaluate(0, out=_outputs(5000, torch.float32))
    torch.cuda.synchronize()
    assert torch.equal(a[0], b[0]) and torch.equal(a[1], b[1])
