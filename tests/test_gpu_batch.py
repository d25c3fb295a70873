"""Batched compression (one chain of launches for many jobs) through the C ABI:
every job's outputs equal the CPU oracle's bit for bit, and equal those of a
plain per-job compression; plans replay through a HIP graph; the autotuner's
choice changes no output."""
import numpy as np
import pytest
import torch

import oracle
from gpu_util import assert_matches_oracle, assert_same_compression, to_np
from paper_1703_02438_amd import inputs
from pins import adversarial_case, mixture_case

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def nk():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_1703_02438_amd.numarck as nk
    return nk


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")


def _mixed_jobs():
    """Jobs of both element types, every encoder class (B < 8, 8, 8 < B < 16,
    16), empty and one-element inputs, ragged sizes, block sizes, an all-invalid
    input and one whose histogram spills out of the window."""
    spec = [
        (0, np.float64, 1e-3, 8, 0), (1, np.float32, 1e-3, 3, 0),
        (100003, np.float64, 1e-3, 10, 0), (4097, np.float32, 1e-2, 1, 0),
        (33, np.float64, 1e-3, 16, 0), (250000, np.float32, 1e-4, 12, 0),
        (65536, np.float64, 1e-3, 8, 4096), (12289, np.float32, 1e-3, 8, 1 << 20),
        (77777, np.float64, 1e-4, 13, 0), (5, np.float64, 1e-3, 5, 0),
        (131071, np.float64, 1e-5, 16, 0), (3, np.float32, 1e-3, 16, 0),
    ]
    jobs = []
    for i, (n, dt, E, B, bb) in enumerate(spec):
        p, q = mixture_case(max(n, 1), 3000 + i, dt)
        jobs.append((p[:n], q[:n], E, B, bb))
    pa, qa = adversarial_case(np.float64)
    pm, qm = mixture_case(20000, 3100, np.float64)
    jobs.append((np.concatenate([pa, pm, pa]), np.concatenate([qa, qm, qa]), 1e-3, 8, 0))
    z = np.zeros(999, np.float64)
    jobs.append((z, z + 1.0, 1e-3, 8, 0))  # no valid point
    return jobs


# with the reconstruction (the encoder reads both snapshots) and without it
# (the precoded encoder)
RECON = pytest.mark.parametrize("recon", [True, False], ids=["reads_snapshots", "precoded"])


def _run_plan(nk, jobs, graph=False, tune=None, recon=True):
    bj = [nk.BatchJob(_dev(p), _dev(q), E, B, bb) for p, q, E, B, bb in jobs]
    plan = nk.Plan(bj, recon=recon, bin_ids=True, tune=tune)
    if graph:
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s):
            plan.capture(s)
            res = plan.replay(s)
        torch.cuda.current_stream().wait_stream(s)
    else:
        res = plan.run()
    return plan, bj, res


@RECON
def test_mixed_batch_vs_oracle(nk, recon):
    jobs = _mixed_jobs()
    plan, bj, res = _run_plan(nk, jobs, recon=recon)
    torch.cuda.synchronize()
    orc = oracle.get()
    for i, ((p, q, E, B, bb), c) in enumerate(zip(jobs, res)):
        o = orc.compress(p, q, E, B, block_bytes=bb)
        assert_matches_oracle(nk, c, o, p, q, E, B, bb, check_hist=False, label=f"job{i}")
        out, fl = nk.decompress(c, bj[i].prev)
        ref, rfl = orc.decompress(o, p)
        assert int(fl.item()) == rfl == 0
        assert np.array_equal(to_np(out).view(np.uint8), ref.view(np.uint8)), f"job{i} decode"
    plan.close()


def test_plan_mixing_both_encoders(nk):
    """Jobs with and without a reconstruction in one plan: the plan keeps the
    two encodings in separate encoder launches, and every job equals the
    oracle (its reconstruction too, where asked for)."""
    jobs = _mixed_jobs()
    bj = [nk.BatchJob(_dev(p), _dev(q), E, B, bb) for p, q, E, B, bb in jobs]
    outs = [nk.alloc_outputs(max(j.prev.numel(), 0), j.prev.dtype, j.B, j.block_bytes,
                             recon=(i % 2 == 0), bin_ids=True) for i, j in enumerate(bj)]
    plan = nk.Plan(bj, outputs=outs)
    enc = [g for g in plan.groups() if g["pass"] == "encode"]
    assert sum(g["njobs"] for g in enc) == len(bj)
    keys = [(g["dtype"], g["cls"]) for g in enc]
    assert len(keys) > len(set(keys)), enc  # a class split by encoding
    res = plan.run()
    torch.cuda.synchronize()
    orc = oracle.get()
    for i, ((p, q, E, B, bb), c) in enumerate(zip(jobs, res)):
        assert (c.recon is not None) == (i % 2 == 0)
        o = orc.compress(p, q, E, B, block_bytes=bb)
        assert_matches_oracle(nk, c, o, p, q, E, B, bb, check_hist=False, label=f"mixed job{i}")
    plan.close()


@RECON
def test_batch_selected_tail_bins(nk, recon):
    """Selected bins on both sides of the window in jobs of one batch: with
    k <= 1024 (B = 8, 10) k_select ranks them, with larger k (B = 12, 16)
    k_tailrank does, in the same launches; every job equals the oracle."""
    rng = np.random.default_rng(77)
    jobs = []
    for i, (B, dt) in enumerate([(8, np.float64), (12, np.float64), (10, np.float32),
                                 (16, np.float32), (8, np.float32)]):
        n = 150_000 + 1000 * i
        prev = rng.lognormal(0, 1, n)
        u = rng.random(n)
        r = np.where(u < 0.3, rng.normal(0, 1e-5, n),
                     np.where(u < 0.5, rng.normal(0.4, 3e-5, n),
                              np.where(u < 0.7, rng.normal(-0.45, 3e-5, n),
                                       rng.uniform(-0.5, 0.5, n))))
        jobs.append((prev.astype(dt), (prev * (1 + r)).astype(dt), 1e-5, B, 0))
    plan, bj, res = _run_plan(nk, jobs, recon=recon)
    torch.cuda.synchronize()
    orc = oracle.get()
    for i, ((p, q, E, B, bb), c) in enumerate(zip(jobs, res)):
        o = orc.compress(p, q, E, B, block_bytes=bb)
        h = c.header()
        ids = o.sel_ids
        assert (ids < h.window_base).any() and (ids >= h.window_base + 16384).any(), i
        assert_matches_oracle(nk, c, o, p, q, E, B, bb, check_hist=False, label=f"tail job{i}")
    plan.close()


@RECON
def test_batch_equals_plain_and_one_shot(nk, recon):
    jobs = _mixed_jobs()
    plan, bj, res = _run_plan(nk, jobs, recon=recon)
    one = nk.compress_batch(bj, recon=recon, bin_ids=True)
    for i, (j, c, c1) in enumerate(zip(bj, res, one)):
        plain = nk.compress(j.prev, j.curr, j.E, j.B, j.block_bytes, recon=recon, bin_ids=True)
        assert_same_compression(c, plain, f"plan vs plain job{i}")
        assert_same_compression(c1, plain, f"one-shot vs plain job{i}")
    plan.close()


@RECON
def test_graph_replays(nk, recon):
    """A captured plan replays several times, with eager work and new input
    values between replays; every replay matches the oracle on what the
    inputs held at that time."""
    jobs = _mixed_jobs()[:6]
    plan, bj, res = _run_plan(nk, jobs, graph=True, recon=recon)
    torch.cuda.synchronize()
    orc = oracle.get()
    s = torch.cuda.Stream()
    for rep in range(3):
        if rep:
            for i, j in enumerate(bj):  # new current snapshots, written in place
                n = j.curr.numel()
                if n == 0:
                    continue
                _, q = mixture_case(n, 5000 + 31 * rep + i,
                                    np.float32 if j.curr.dtype == torch.float32 else np.float64)
                j.curr.copy_(_dev(q))
            junk = torch.randn(1 << 20, device="cuda").sum()  # eager work between replays
            torch.cuda.synchronize()
            s.wait_stream(torch.cuda.current_stream())
            with torch.cuda.stream(s):
                res = plan.replay(s)
            s.synchronize()
            del junk
        for i, (j, c) in enumerate(zip(bj, res)):
            p, q = to_np(j.prev), to_np(j.curr)
            o = orc.compress(p, q, j.E, j.B, block_bytes=j.block_bytes)
            assert_matches_oracle(nk, c, o, p, q, j.E, j.B, j.block_bytes, check_hist=False,
                                  label=f"replay{rep} job{i}")
    plan.close()


def test_uneven_variables_batch(nk):
    """The uneven multi-variable workload (log-uniform cube edges, mixed
    float32/float64, E in {1e-4, 1e-3, 1e-2}, B in {8, 10, 12}), 64 variables
    at reduced edges, against the oracle."""
    specs = inputs.batched_specs(64, lo_edge=8, hi_edge=64)
    jobs = []
    for sp in specs:
        p, q = inputs.mixture_pair(sp.n, seed=sp.seed, dtype=sp.dtype)
        jobs.append((p.numpy(), q.numpy(), sp.E, sp.B, 0))
    plan, bj, res = _run_plan(nk, jobs)
    torch.cuda.synchronize()
    orc = oracle.get()
    for i, ((p, q, E, B, bb), c) in enumerate(zip(jobs, res)):
        o = orc.compress(p, q, E, B)
        assert_matches_oracle(nk, c, o, p, q, E, B, check_hist=False, label=f"var{i}")
    plan.close()


def test_time_series_pairs(nk):
    """Sixteen consecutive snapshot pairs of one climate-like series in one
    batch (pairs share snapshots), against the oracle."""
    s = inputs.ClimateSeries(nlat=90, nlon=180, seed=1708, device="cuda")
    snaps = [s.x.clone()]
    for _ in range(16):
        snaps.append(s.step().clone())
    bj = [nk.BatchJob(snaps[t], snaps[t + 1], 1e-4, 10) for t in range(16)]
    plan = nk.Plan(bj, recon=True, bin_ids=True)
    res = plan.run()
    torch.cuda.synchronize()
    orc = oracle.get()
    for t, c in enumerate(res):
        p, q = to_np(snaps[t]), to_np(snaps[t + 1])
        o = orc.compress(p, q, 1e-4, 10)
        assert_matches_oracle(nk, c, o, p, q, 1e-4, 10, check_hist=False, label=f"pair{t}")
    plan.close()


def test_tunings_change_no_output(nk):
    p, q = mixture_case(300001, 4242, np.float64)
    P, Q = _dev(p), _dev(q)
    ref = nk.compress(P, Q, 1e-3, 8, recon=True, bin_ids=True)
    for rb, hb, hl, cv, up, sl in [(1, 1, 1, 64, 1, 1), (16, 4, 0, 16384, 50, 2),
                                   (64, 16, 0, 1 << 20, 100, 0), (3, 2, 1, 777, 33, 1)]:
        t = nk.NumarckTuning(rb, hb, hl, cv, up, sl)
        c = nk.compress_tuned(P, Q, 1e-3, 8, t)
        assert_same_compression(c, ref, f"tuning {t.as_dict()}")
        plan, _, res = _run_plan(nk, [(p, q, 1e-3, 8, 0)], tune=t)
        assert_same_compression(res[0], ref, f"plan tuning {t.as_dict()}")
        plan.close()


def test_autotune(nk, tmp_path):
    p, q = mixture_case(1 << 20, 4343, np.float32)
    P, Q = _dev(p), _dev(q)
    best = nk.autotune(P, Q, 1e-3, 8, reps=2)
    d = best.as_dict()
    assert 1 <= d["unit_pct"] <= 100 and d["hist_lds"] in (0, 1)
    c = nk.compress(P, Q, 1e-3, 8, recon=True, bin_ids=True)  # uses the recorded tuning
    o = oracle.get().compress(p, q, 1e-3, 8)
    assert_matches_oracle(nk, c, o, p, q, 1e-3, 8, check_hist=False, label="autotuned")
    path = str(tmp_path / "tune.txt")
    assert nk.numarck_tuning_save(path.encode()) == nk.OK
    assert "f32 20 " in open(path).read()
    assert nk.numarck_tuning_load(path.encode()) == nk.OK


def _series(n, dt, seed, steps, E=1e-3):
    rng = np.random.default_rng(seed)
    x = rng.lognormal(0.0, 1.0, n)
    x[rng.choice(n, max(1, n // 500), replace=False)] = 0.0  # invalid points
    out = [x.astype(dt)]
    for _ in range(steps):
        u = rng.random(n)
        r = np.where(u < 0.8, rng.normal(0, 2 * E, n), rng.uniform(-0.3, 0.3, n))
        out.append((out[-1].astype(np.float64) * (1 + r)).astype(dt))
    return [_dev(a) for a in out]


def test_time_chains(nk):
    """Batches whose range pass sweeps time chains (each job's prev is the
    previous job's curr): ragged lengths with a scalar remainder, both element
    types, a chain longer than one sweep takes (cut in two), a chain broken by
    another snapshot, per-pair error bounds, and unchained jobs between
    chains.  Every job equals its plain compression; some equal the oracle."""
    fa = _series(100_003, np.float64, 51, 6)
    fb = _series(262_147, np.float32, 52, 5)
    fc = _series(4_099, np.float32, 53, 70)  # 70 pairs: more than one chain
    other = _series(100_003, np.float64, 54, 1)
    jobs = []
    for t in range(3):
        jobs.append((fa[t], fa[t + 1], 1e-3 * (t + 1), 8))
    jobs.append((other[0], other[1], 1e-3, 8))  # breaks the chain of fa
    for t in range(3, 6):
        jobs.append((fa[t], fa[t + 1], 1e-4, 12))
    for t in range(5):
        jobs.append((fb[t], fb[t + 1], 1e-3, 10))
    for t in range(70):
        jobs.append((fc[t], fc[t + 1], 1e-2, 5))
    bj = [nk.BatchJob(p, q, E, B) for p, q, E, B in jobs]
    plan = nk.Plan(bj, recon=True, bin_ids=True)
    for rep in range(2):
        res = plan.run()
        torch.cuda.synchronize()
        for i, ((p, q, E, B), c) in enumerate(zip(jobs, res)):
            ref = nk.compress(p, q, E, B, recon=True, bin_ids=True)
            assert_same_compression(c, ref, f"job {i} rep {rep}")
    orc = oracle.get()
    for i in (0, 5, 8, 80):
        p, q, E, B = jobs[i]
        pn, qn = to_np(p), to_np(q)
        assert_matches_oracle(nk, res[i], orc.compress(pn, qn, E, B), pn, qn, E, B,
                              check_hist=False, label=f"chain job {i}")
    plan.close()


def test_plan_autotune(nk):
    """numarck_plan_autotune on a batch of many small uneven jobs (where the
    histogram's placement is a real choice) returns a valid tuning; a plan
    built with it gives every job's plain compression bit for bit, for both
    anchorings."""
    specs = inputs.batched_specs(48, seed=1719, lo_edge=8, hi_edge=48)
    pairs = [inputs.mixture_pair(sp.n, seed=sp.seed, dtype=sp.dtype, device="cuda")
             for sp in specs]
    bj = [nk.BatchJob(p, q, sp.E, sp.B) for (p, q), sp in zip(pairs, specs)]
    for za in (False, True):
        best = nk.plan_autotune(bj, reps=2, zero_anchored=za)
        d = best.as_dict()
        assert d["hist_lds"] in (0, 1) and 1 <= d["unit_pct"] <= 100, d
        assert 1 <= d["range_blocks_per_cu"] <= 8 and 1 <= d["hist_blocks_per_cu"] <= 8, d
        plan = nk.Plan(bj, recon=True, bin_ids=True, tune=best, zero_anchored=za)
        res = plan.run()
        torch.cuda.synchronize()
        plain = nk.compress_zero_anchored if za else nk.compress
        for i, ((p, q), sp, c) in enumerate(zip(pairs, specs, res)):
            ref = plain(p, q, sp.E, sp.B, recon=True, bin_ids=True)
            assert_same_compression(c, ref, f"autotuned plan za={za} job {i} {d}")
        plan.close()
