"""GPU: spd_search_noalloc (the library's fixed device workspace) against spd_search with a
workspace of the caller's, through the C ABI, on two calls in a row (the second smaller)."""
import sys

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no ROCm device")
    from paper_1910_08324_amd import spd
    spd.load()
    return torch.device("cuda:0")


def inputs(dev, n_dm, n, seed):
    rng = np.random.default_rng(seed)
    mu = rng.uniform(-1, 1, n_dm).astype(np.float32)
    sg = rng.uniform(0.5, 2.0, n_dm).astype(np.float32)
    x = synth.noise_rows(n, seed, range(n_dm)) * sg[:, None] + mu[:, None]
    synth.inject(x, [synth.Pulse(n_dm // 2, n // 3, 37, 25.0 * float(sg[n_dm // 2])),
                     synth.Pulse(1, n // 2, 300, 30.0 * float(sg[1]), "gauss")])
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to(dev)
    return t(x), t(mu), t(sg)


def same(a, b):
    from paper_1910_08324_amd import spd
    for i in range(a.info.n_levels):
        Ya, Wa = a.level(i)
        Yb, Wb = b.level(i)
        assert torch.equal(Ya, Yb), f"level {i} snr"
        assert torch.equal(Wa, Wb), f"level {i} width"


@pytest.mark.parametrize("method,l_end,planes", [("ig1", 8192, True), ("bd16", 1024, True),
                                                 ("ig2", 512, False), ("exh", 300, True)])
def test_noalloc_equals_search(dev, method, l_end, planes):
    from paper_1910_08324_amd import spd
    cfg = spd.Config(method, l_end, threshold=4.5, planes=planes)
    # two calls in a row on the same stream, the second on a smaller input
    for (n_dm, n, seed) in ((96, 40000 + 4 * l_end, 11), (17, 5003, 12)):
        say(f"noalloc {method} L_end {l_end} planes={planes}: {n_dm} x {n}")
        x, mu, sg = inputs(dev, n_dm, n, seed)
        ref = spd.search(x, mu, sg, cfg, cand_cap=1 << 14)
        out = spd.search(x, mu, sg, cfg, cand_cap=1 << 14)      # output buffers of the same shape
        if planes:
            out.snr.fill_(7.0)
            out.width.fill_(3)
        out.cand.fill_(0)
        out.count.fill_(-1)
        spd.search_noalloc(x, mu, sg, cfg, out)
        torch.cuda.synchronize()
        if planes:
            same(ref, out)
        nc = int(ref.count.item())
        assert int(out.count.item()) == nc
        assert nc > 0
        assert np.array_equal(ref.candidates_host(), out.candidates_host())


def test_noalloc_rejects_oversize_before_any_launch(dev):
    from paper_1910_08324_amd import spd
    cfg = spd.Config("ig1", 8192)
    n_dm, n = 4096, 262144
    info = spd.plan(cfg, n_dm, n)
    assert info.workspace_bytes > spd.NOALLOC_SCRATCH_BYTES
    x = torch.empty((n_dm, 8), dtype=torch.float32, device=dev)   # never read: rejected first
    mu = torch.zeros(n_dm, dtype=torch.float32, device=dev)
    out = spd.Result(info, None, None, torch.empty(24, dtype=torch.uint8, device=dev),
                     torch.zeros(1, dtype=torch.int64, device=dev), n_dm)
    cfg2 = spd.Config("ig1", 8192, planes=False)
    p, keep = cfg2.params()
    lib = spd.load()
    import ctypes
    st = lib.spd_search_noalloc(ctypes.byref(p), ctypes.c_void_p(x.data_ptr()), n, n_dm, n, n,
                                0, ctypes.c_void_p(mu.data_ptr()), ctypes.c_void_p(mu.data_ptr()),
                                None, None, ctypes.c_void_p(out.cand.data_ptr()), 1,
                                ctypes.c_void_p(out.count.data_ptr()),
                                ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert st == spd.SPD_EWORKSPACE
