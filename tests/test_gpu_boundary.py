"""GPU checks of the C-ABI's resource and persistence calls: the device-memory
hook (fmm_set_allocator) and the cost-model file (fmm_costmodel_save/load)."""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _inputs(n=12000, seed=51):
    x, y, z = synth.plummer(n, seed)
    q = synth.charges_uniform(n, 100 + seed)
    return [torch.tensor(np.asarray(a, np.float32), device="cuda:0") for a in (x, y, z, q)]


def _run(f, t, p=8, theta=0.5, ncrit=32):
    f.build_tree(*t, ncrit)
    f.traverse(p, theta, 0)
    phi, E = f.evaluate()
    torch.cuda.synchronize()
    return phi.cpu().numpy(), E.cpu().numpy()


def test_allocator_hook_failure_is_out_of_memory_and_context_survives():
    from paper_1108_5815_amd import FMM, FMMError
    t = _inputs()
    ref_phi, ref_E = _run(FMM(0), t)
    f = FMM(0)
    calls = []
    f.set_allocator(lambda n: calls.append(n) or 0, lambda ptr: None)
    with pytest.raises(FMMError) as e:
        f.build_tree(*t, 32)
    assert e.value.status == 2 and calls
    with pytest.raises(FMMError) as e:      # the failed build left no tree
        f.traverse(8, 0.5, 0)
    assert e.value.status == 4
    f.set_allocator(None, None)
    phi, E = _run(f, t)
    assert np.array_equal(phi, ref_phi) and np.array_equal(E, ref_E)


def test_allocator_hook_serves_every_buffer():
    """Through a counting hook over torch's caching allocator the results are
    bit-identical, and destroying the context returns every block."""
    from paper_1108_5815_amd import FMM
    t = _inputs()
    ref_phi, ref_E = _run(FMM(0), t)
    live = {}
    f = FMM(0)

    def alloc(n):
        ptr = torch.cuda.caching_allocator_alloc(n, 0)
        live[ptr] = n
        return ptr

    def free(ptr):
        del live[ptr]
        torch.cuda.caching_allocator_delete(ptr)

    f.set_allocator(alloc, free)
    phi, E = _run(f, t)
    assert np.array_equal(phi, ref_phi) and np.array_equal(E, ref_E)
    assert len(live) > 10 and all(ptr % 256 == 0 for ptr in live)
    # a second, larger problem grows buffers: old blocks go back through the hook
    t2 = _inputs(30000, 52)
    _run(f, t2)
    f.close()
    assert live == {}


def test_allocator_hook_needs_both_routines():
    import ctypes
    from paper_1108_5815_amd import FMM
    from paper_1108_5815_amd.binding import ALLOC_FN, lib
    f = FMM(0)
    a = ALLOC_FN(lambda n, u: None)
    assert lib().fmm_set_allocator(f.h, ctypes.cast(a, ctypes.c_void_p), None, None) == 1


def _records(seed=3, n=600):
    rng = np.random.default_rng(seed)
    feat = rng.uniform(-1, 1, (n, 6)).astype(np.float32)
    kind = rng.integers(0, 3, n).astype(np.int32)
    tgt = (feat[:, 1] * 3 + kind + feat[:, 2] * (kind == 2)).astype(np.float32)
    return feat, kind, tgt


def test_costmodel_save_load_roundtrip(tmp_path):
    from paper_1108_5815_amd import FMM, FMMError
    f = FMM(0)
    with pytest.raises(FMMError) as e:
        f.costmodel_save(str(tmp_path / "none.txt"))
    assert e.value.status == 4
    f.costmodel_fit(*_records(), epochs=200, lr=3e-3, seed=5)
    f.set_costs(0.4, 0.3, 0.001)
    f.set_tile_config([1, 2, -2, 4])
    f.set_overlap(1)
    f.set_m2l_kernel(3)
    f.set_m2l_tile(128)
    path = str(tmp_path / "cm.txt")
    f.costmodel_save(path)
    g = FMM(0)
    g.costmodel_load(path)                     # any p, any precision
    assert np.array_equal(g.costmodel_weights(), f.costmodel_weights())
    assert np.array_equal(g.costs(), f.costs())
    assert g.tile_config() == {"p2p_targets_per_lane": [1, 2, -2, 4], "schedule": 1, "m2l_kernel": 3, "m2l_tile": 128}
    assert np.array_equal(g.costmodel_table(10, 0.4), f.costmodel_table(10, 0.4))
    text = open(path).read()
    assert text.startswith("fmm-costmodel 1\n") and "\np -1\n" in text
    # keyed by order and precision: the fitted model records neither
    with pytest.raises(FMMError) as e:
        g.costmodel_load(path, p=10)
    assert e.value.status == 1
    # another device's model, or a damaged file, is refused and the model kept
    w0 = g.costmodel_weights()
    lines = text.split("\n")
    lines[1] = "device gfx000/1cu"
    open(tmp_path / "other.txt", "w").write("\n".join(lines))
    bad_weights = text.replace("\nend\n", "\n")
    bad_weights = bad_weights[:len(bad_weights) // 2]
    open(tmp_path / "cut.txt", "w").write(bad_weights)
    open(tmp_path / "v2.txt", "w").write(text.replace("fmm-costmodel 1", "fmm-costmodel 2", 1))
    for name in ("other.txt", "cut.txt", "v2.txt", "missing.txt"):
        with pytest.raises(FMMError) as e:
            g.costmodel_load(str(tmp_path / name))
        assert e.value.status == 1, name
    assert np.array_equal(g.costmodel_weights(), w0)


def test_costmodel_trained_file_keys(tmp_path):
    """A model trained by the library records its order, theta and precision,
    and loads only for them."""
    from paper_1108_5815_amd import FMM, FMMError
    f = FMM(0)
    f.costmodel_train(6, 0.5, epochs=50, seed=3, precision=0)
    path = str(tmp_path / "cm6.txt")
    f.costmodel_save(path)
    text = open(path).read()
    assert "\np 6\n" in text and "\nprecision 0\n" in text
    g = FMM(0)
    g.costmodel_load(path, p=6, precision=0)
    assert np.array_equal(g.costmodel_weights(), f.costmodel_weights())
    with pytest.raises(FMMError):
        g.costmodel_load(path, p=6, precision=1)
