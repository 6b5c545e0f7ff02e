"""Concurrent calls on different streams.

The library's handles are immutable after creation, so sampling calls and
kernel tabulations on different streams may run at the same time (bench.py
tabulates the next step's kernels on a second stream while the current step
samples).  Results must be bitwise equal to the same calls made one after
another on one stream.
"""
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import paper_1504_04653_amd as sp
from workloads import synth as S

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module", autouse=True)
def gpu():
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    torch.cuda.set_device(0)
    yield
    torch.cuda.synchronize()


def test_concurrent_streams_match_sequential_calls():
    lmax = 256
    g = sp.Grid(lmax, 8)
    rng = np.random.default_rng(77)
    ninv = torch.as_tensor(rng.uniform(0.5, 2.0, g.npix)).cuda()
    b_l, R = S.gaussian_beam(lmax, g.npix, 3.0)
    d_l = S.prior(lmax)
    b2_l, R2 = S.gaussian_beam(lmax, g.npix, 4.0)
    new = lambda: torch.full((g.out_len,), float("nan"), dtype=torch.float64, device="cuda")

    # sequential reference on the current stream
    kb = sp.Kernel(g, b_l, R)
    kd = sp.Kernel(g, d_l, 0.0)
    kb2 = sp.Kernel(g, b2_l, R2)
    D0, C0, F0, E0 = new(), new(), new(), new()
    sp.sample_D_BtNB(g, kd, kb, ninv, D0, C0, "bf16x6")
    sp.sample_BtNB(g, kb, ninv, F0, "fp64")
    sp.sample_BtNB(g, kb2, ninv, E0, "fp32")
    torch.cuda.synchronize()

    # the same work on three streams, started together
    s1, s2, s3 = torch.cuda.Stream(), torch.cuda.Stream(), torch.cuda.Stream()
    D1, C1, F1, E1 = new(), new(), new(), new()
    torch.cuda.synchronize()
    with torch.cuda.stream(s1):
        kb2b = sp.Kernel(g, b2_l, R2, stream=s1)                         # a tabulation ...
        sp.sample_BtNB(g, kb2b, ninv, E1, "fp32", stream=s1)
    with torch.cuda.stream(s2):
        sp.sample_D_BtNB(g, kd, kb, ninv, D1, C1, "bf16x6", stream=s2)   # ... beside sampling
    with torch.cuda.stream(s3):
        sp.sample_BtNB(g, kb, ninv, F1, "fp64", stream=s3)              # with a shared handle
    torch.cuda.synchronize()
    for name, a, b in (("D-hat", D1, D0), ("bf16x6", C1, C0), ("fp64", F1, F0), ("fp32", E1, E0)):
        assert torch.equal(a, b), f"{name}: concurrent result differs from the sequential one"
    say(f"[streams] lmax {lmax}: four results on three streams bitwise equal to sequential calls")
    del kb2b
