"""GPU parity of batched launches: many B-hat^T N^-1 B-hat problems (FP64,
FP32 or split-BF16 MFMA; the latter two with FP64 accumulation across
contraction tiles) in one captured graph.

Every schedule must give results bitwise identical to the single-problem path
of the same mode (each work item is computed by the same arithmetic whichever
workgroup takes it), and those results must meet the mode's gate against the
oracle.  Graph replays are checked with eager work and synchronisations in
between.
"""
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import paper_1504_04653_amd as sp
from oracle import grid as G
from oracle import operators as O
from workloads import synth as S

from _parity import block_index, error_report, stored_pairs

pytestmark = pytest.mark.gpu

GATE = {"fp64": 1e-10, "fp32": 1e-6, "bf16x6": 1e-6, "bf16x3": 2.0 ** -15}
BATCH_MODES = ["fp64", "fp32", "bf16x6", "bf16x3"]

# (lmax, problem index whose beam / mask draws are used): mixed sizes, with
# two problems on one grid
SMALL = [(64, 0), (128, 1), (64, 2), (256, 3), (96, 4), (160, 5)]


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module", autouse=True)
def gpu():
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    torch.cuda.set_device(0)
    yield
    torch.cuda.synchronize()
    torch.cuda.empty_cache()


def dev(x):
    return torch.as_tensor(np.ascontiguousarray(x, dtype=np.float64)).cuda()


def make_problems(spec):
    grids, probs = {}, []
    for lmax, p in spec:
        if lmax not in grids:
            grids[lmax] = (G.make_grid(lmax, 8), sp.Grid(lmax, 8))
        og, g = grids[lmax]
        prob = dict(S.batch_problem(p))
        prob["lmax"] = lmax
        ring, _, _, phi = og.pixel_coords()
        ninv = S.ninv_batch(og.theta[ring], phi, prob)
        b_l, R = S.gaussian_beam(lmax, g.npix, prob["fwhm_pix"])
        probs.append(dict(og=og, g=g, ninv=ninv, b_l=b_l, R=R, kb=sp.Kernel(g, b_l, R),
                          ninv_dev=dev(ninv),
                          out=torch.empty(g.out_len, dtype=torch.float64, device="cuda")))
    return probs


def single(p, prec):
    out = torch.empty(p["g"].out_len, dtype=torch.float64, device="cuda")
    sp.sample_BtNB(p["g"], p["kb"], p["ninv_dev"], out, prec)
    torch.cuda.synchronize()
    return out


@pytest.fixture(scope="module")
def problems():
    probs = make_problems(SMALL)
    say("[batch] problems " + ", ".join(f"lmax {p['g'].lmax}: {p['g'].nblocks} blocks" for p in probs))
    return probs


@pytest.fixture(scope="module", params=BATCH_MODES)
def small(request, problems):
    prec = request.param
    probs = problems
    bt = sp.Batch([(p["g"], p["kb"], p["ninv_dev"], p["out"]) for p in probs], prec=prec)
    ref = [single(p, prec) for p in probs]
    yield dict(probs=probs, bt=bt, ref=ref, prec=prec)
    bt.close()


def launch_and_check(small, tag):
    for p in small["probs"]:
        p["out"].fill_(float("nan"))
    torch.cuda.synchronize()
    small["bt"].launch()
    torch.cuda.synchronize()
    for i, (p, r) in enumerate(zip(small["probs"], small["ref"])):
        assert torch.equal(p["out"], r), f"{tag}: problem {i} differs from the single-problem {small['prec']} path"


@pytest.mark.parametrize("tiling", ["tiles64", "tiles32"])
@pytest.mark.parametrize("schedule", ["xcd_queues", "global_lpt", "per_problem"])
def test_every_schedule_matches_single_problem_path(small, schedule, tiling):
    small["bt"].set_tiling(tiling)
    small["bt"].set_schedule(schedule)
    launch_and_check(small, f"{schedule}/{tiling}")
    say(f"[batch {small['prec']}] {schedule}/{tiling}: bitwise equal to sample_BtNB for {len(small['probs'])} problems")


def test_single_problem_path_against_oracle(small):
    for i, (p, r) in enumerate(zip(small["probs"], small["ref"])):
        pairs = stored_pairs(p["og"])
        rows = [J for J, _ in pairs]
        Cref = O.sample_BtNB(p["og"], p["b_l"], p["ninv"], p["R"], pairs)
        rep = error_report(r.view(-1, 64, 64).cpu().numpy(), Cref, rows)
        say(f"[batch {small['prec']}] problem {i} lmax {p['g'].lmax}: {rep}")
        assert rep["gate"] <= GATE[small["prec"]]


def test_graph_replays_with_eager_work_between(small):
    small["bt"].set_tiling("tiles64")
    small["bt"].set_schedule("xcd_queues")
    for r in range(3):
        x = torch.randn(1 << 20, device="cuda", dtype=torch.float64)
        s = float((x * x).sum())           # eager kernels and a host sync between replays
        assert s > 0
        launch_and_check(small, f"replay {r}")


def test_tune_picks_a_plan_and_keeps_results(small):
    chosen, ms = small["bt"].tune()
    say(f"[batch {small['prec']}] tune: chosen {sp.plan_name(chosen)}, ms per plan {ms}")
    assert len(ms) == len(sp.SCHEDULES) * len(sp.TILINGS)
    assert chosen in range(len(ms))
    assert all(t > 0 for t in ms)
    assert ms[chosen] == min(ms)
    launch_and_check(small, "after tune")


def test_launch_then_retune_on_a_side_stream(small):
    """A launch queued on a non-blocking stream, followed at once by a tile
    shape change, a schedule change and a tune (each re-captures the graph
    and rewrites the work-item tables): the re-capture waits for the launch,
    and every result stays bitwise equal to the single-problem path."""
    side = torch.cuda.Stream()
    for p in small["probs"]:
        p["out"].fill_(float("nan"))
    torch.cuda.synchronize()
    small["bt"].set_tiling("tiles64")
    small["bt"].set_schedule("xcd_queues")
    small["bt"].launch(side)
    small["bt"].set_tiling("tiles32")           # no host synchronisation in between
    small["bt"].launch(side)
    small["bt"].set_schedule("global_lpt")
    small["bt"].launch(side)
    small["bt"].tune(side)
    side.synchronize()
    for i, (p, r) in enumerate(zip(small["probs"], small["ref"])):
        assert torch.equal(p["out"], r), f"problem {i} differs after launch-then-retune on a side stream"
    launch_and_check(small, "after retune")
    say(f"[batch {small['prec']}] launch / re-capture / tune on a side stream: results unchanged")


def test_batch_argument_errors(small):
    p = small["probs"][0]
    q = small["probs"][2]                   # same grid as p
    with pytest.raises(sp.SympixError) as ei:
        sp.Batch([(p["g"], p["kb"], p["ninv_dev"], p["out"])], prec=7)
    assert ei.value.code == "EINVAL"
    buf = torch.zeros(p["g"].npix + 8, dtype=torch.float64, device="cuda")
    off = 1 if (buf.data_ptr() // 8) % 4 == 0 else 0          # an 8-byte but not 32-byte aligned view
    misaligned = buf[off:off + p["g"].npix]
    assert misaligned.data_ptr() % 32 != 0
    with pytest.raises(sp.SympixError) as ei:                  # FP64 reads N^-1 in 32-byte vectors
        sp.Batch([(p["g"], p["kb"], misaligned, p["out"])], prec="fp64")
    assert ei.value.code == "EINVAL"
    short = torch.empty(p["g"].out_len - 1, dtype=torch.float64, device="cuda")
    with pytest.raises(sp.SympixError) as ei:
        sp.Batch([(p["g"], p["kb"], p["ninv_dev"], short)])
    assert ei.value.code == "ESIZE"
    with pytest.raises(sp.SympixError) as ei:
        sp.Batch([(p["g"], p["kb"], p["ninv_dev"], p["out"]), (q["g"], q["kb"], q["ninv_dev"], p["out"])])
    assert ei.value.code == "EINVAL"
    other = small["probs"][1]               # kernel of another grid
    with pytest.raises(sp.SympixError) as ei:
        sp.Batch([(p["g"], other["kb"], p["ninv_dev"], p["out"])])
    assert ei.value.code == "EINVAL"
    for bad in (lambda: small["bt"].set_schedule(3), lambda: small["bt"].set_tiling(2)):
        with pytest.raises(sp.SympixError) as ei:
            bad()
        assert ei.value.code == "EINVAL"


# --- the 32-problem batch at full size, sampled block-rows --------------------

def c5_rows(og, seed):
    """Block-rows compared per problem: the first tile of the polar band, of
    the first band whose tile count differs from a neighbour's and of an
    equatorial band, and one random tile."""
    rng = np.random.default_rng(seed)
    nb = len(og.band_tiles)
    trans = [b for b in range(nb) if any(og.band_tiles[x] != og.band_tiles[b] for x in og.band_neighbours(b))]
    rows = {0, int(og.band_tile0[trans[0]]) if trans else 0, int(og.band_tile0[nb - 1]),
            int(rng.integers(og.ntiles))}
    return sorted(rows)


@pytest.mark.parametrize("prec", ["fp32", "bf16x6", "fp64"])
def test_c5_full_batch_sampled(prec):
    spec = [(S.BATCH_LMAX[p % 4], p) for p in range(32)]
    probs = make_problems(spec)
    total = sum(p["g"].nblocks for p in probs) * 4096 * 8
    say(f"[batch32 {prec}] 32 problems, {sum(p['g'].npix for p in probs)} pixels, output {total / 1e9:.1f} GB")
    bt = sp.Batch([(p["g"], p["kb"], p["ninv_dev"], p["out"]) for p in probs], prec=prec)
    chosen, ms = bt.tune()
    say(f"[batch32 {prec}] tune: chosen {sp.plan_name(chosen)}, ms per plan {[round(t, 2) for t in ms]}")
    for p in probs:
        p["out"].fill_(float("nan"))
    bt.launch()
    torch.cuda.synchronize()
    worst = 0.0
    for i, p in enumerate(probs):
        og, g = p["og"], p["g"]
        rows = c5_rows(og, seed=7000 + i)
        brp, bcol = g.blocks()
        idx, pairs = block_index(og, brp, bcol, rows)
        op = O.LocalOperator(og, p["b_l"], p["R"])
        Cref = np.stack([O.btnb_block(op, p["ninv"], J, K) for J, K in pairs])
        C = p["out"].view(-1, 64, 64)[torch.as_tensor(idx, device="cuda")].cpu().numpy()
        rep = error_report(C, Cref, [J for J, _ in pairs])
        worst = max(worst, rep["gate"])
        say(f"[batch32 {prec}] problem {i} lmax {g.lmax}: {len(idx)} blocks, {rep}")
        assert rep["gate"] <= GATE[prec]
        assert not bool(torch.isnan(p["out"]).any()), f"problem {i}: a block was not written"
    say(f"[batch32 {prec}] worst gate {worst:.3e}")
    bt.close()
    for p in probs:
        del p["out"]
    torch.cuda.empty_cache()


TUNE_SCRIPT = r"""
import sys
import numpy as np
import torch
import paper_1504_04653_amd as sp
from workloads import synth as S
torch.cuda.set_device(0)
keep = []
for lmax, p in ((64, 0), (128, 1)):
    g = sp.Grid(lmax, 8)
    b_l, R = S.gaussian_beam(lmax, g.npix, 3.0)
    kb = sp.Kernel(g, b_l, R)
    n = torch.as_tensor(np.random.default_rng(p).uniform(0.5, 2.0, g.npix)).cuda()
    out = torch.empty(g.out_len, dtype=torch.float64, device="cuda")
    keep.append((g, kb, n, out))
bt = sp.Batch(keep, prec="fp32")
if sys.argv[1] == "tune":
    chosen, _ = bt.tune()
    print("PLAN", chosen, flush=True)
else:
    print("PLAN", bt.plan(), flush=True)
bt.close()
"""


def test_tuner_cache_file_carries_the_plan_to_another_process(tmp_path):
    """SYMPIX_TUNE_CACHE: one process tunes and records its plan in the file;
    a later process creating a batch of the same problems starts from it."""
    import os
    import subprocess
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    cache = tmp_path / "tune.txt"
    env = dict(os.environ, SYMPIX_TUNE_CACHE=str(cache), PYTHONPATH=root)

    def run(mode):
        res = subprocess.run([sys.executable, "-c", TUNE_SCRIPT, mode], capture_output=True, text=True, env=env,
                             timeout=300, cwd=root)
        assert res.returncode == 0, res.stderr[-2000:]
        return int([l for l in res.stdout.splitlines() if l.startswith("PLAN")][0].split()[1])

    chosen = run("tune")
    lines = cache.read_text().splitlines()
    assert len(lines) == 1 and lines[0].endswith("\t%d" % chosen) and "|fp32|" in lines[0]
    assert run("plan") == chosen
    say(f"[batch] tuner cache file: plan {sp.plan_name(chosen)} recorded and picked up by a new process")
