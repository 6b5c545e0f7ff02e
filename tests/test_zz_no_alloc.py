"""GPU test (collected last) of the allocation-free entry point sympix_sample_BtNB_noalloc,
called through the C ABI: in every precision mode its output equals that of
sympix_sample_BtNB (same kernels, N^-1 operands in the library's static device
array instead of a stream-ordered allocation), bit for bit, on two calls in a
row, the second on a smaller grid; a grid beyond the array's limit is refused
before anything is launched."""
import ctypes
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import paper_1504_04653_amd as sp
from workloads import synth as S

pytestmark = pytest.mark.gpu

MODES = ("fp64", "fp32", "bf16x6", "bf16x3")


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module", autouse=True)
def gpu():
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    torch.cuda.set_device(0)
    yield
    torch.cuda.synchronize()


def problem(lmax, seed):
    g = sp.Grid(lmax, 8)
    rng = np.random.default_rng(seed)
    ninv = rng.uniform(0.5, 2.0, g.npix)
    ninv[rng.random(g.npix) < 0.1] = 0.0
    b_l, R = S.gaussian_beam(lmax, g.npix, 3.0)
    kb = sp.Kernel(g, b_l, R)
    n_dev = torch.as_tensor(ninv).cuda()
    return g, kb, n_dev


def noalloc_abi(g, kb, n_dev, out, prec):
    """The entry point through its C signature (raw pointers and lengths)."""
    fn = sp.raw_call("sympix_sample_BtNB_noalloc")
    fn.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32,
                   ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p]
    fn.restype = ctypes.c_int
    st = torch.cuda.current_stream().cuda_stream
    return fn(g.handle, kb.handle, n_dev.data_ptr(), n_dev.numel(), sp.PRECISIONS[prec], out.data_ptr(),
              out.numel(), st)


@pytest.mark.parametrize("prec", MODES)
def test_noalloc_matches_sample_BtNB_on_two_calls(prec):
    big = problem(256, 11)
    small = problem(64, 12)           # second call: fewer pixels, the array keeps the first call's tail
    for tag, (g, kb, n_dev) in (("lmax 256", big), ("lmax 64", small)):
        ref = torch.full((g.out_len,), float("nan"), dtype=torch.float64, device="cuda")
        sp.sample_BtNB(g, kb, n_dev, ref, prec)
        out = torch.full((g.out_len,), float("nan"), dtype=torch.float64, device="cuda")
        torch.cuda.synchronize()
        assert noalloc_abi(g, kb, n_dev, out, prec) == 0, sp.raw_call("sympix_last_error")()
        torch.cuda.synchronize()
        assert not bool(torch.isnan(out).any()), f"{prec} {tag}: a block was not written"
        assert torch.equal(out, ref), f"{prec} {tag}: differs from sample_BtNB"
        say(f"[noalloc {prec}] {tag}: npix {g.npix}, {g.nblocks} blocks, bitwise equal to sample_BtNB")


def test_noalloc_refuses_a_grid_beyond_its_scratch():
    g = sp.Grid(3500, 8)                # 17,575,552 pixels > 2^24
    assert g.npix > (1 << 24)
    kb = sp.Kernel(g, S.gaussian_beam(3500, g.npix, 3.0)[0], 0.0)
    n_dev = torch.ones(g.npix, dtype=torch.float64, device="cuda")
    out = torch.zeros(1, dtype=torch.float64, device="cuda")   # wrong length too: nothing could launch
    with pytest.raises(sp.SympixError) as ei:
        sp.sample_BtNB_noalloc(g, kb, n_dev, out, "bf16x6")
    assert ei.value.code == "ESIZE"
    assert "allocation-free" in str(ei.value)
    assert float(out[0]) == 0.0
    say(f"[noalloc] lmax 3500 ({g.npix} pixels) refused: {ei.value}")
