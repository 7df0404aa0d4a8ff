"""Batching form on the GPU (nfs_batch_*): many sequences of uneven frame
size and length run together on several streams, eagerly or as a replayed
HIP graph, give per sequence exactly what a single plan gives on the same
frames; with a memory budget that forces time-windowed rings they still
match the FP64 oracle."""
import numpy as np
import pytest
import torch

import gen
import oracle
from gpu_util import assert_D_close, require_gpu, say

pytestmark = pytest.mark.gpu


def _small_batch(count=6, seed=7):
    return gen.batch_workload(master_seed=seed, count=count, sizes=(32, 64, 128),
                              frames=(20, 90), lag_count=8)


def _seq(c, capacity=None):
    return dict(n=c["n"], lags=c["lags"], n_bins=c["n_bins"], in_dtype="u16",
                capacity=capacity or max(c["N"], c["lags"][-1] + 1))


def _single(c, frames):
    import paper_1209_3362_amd as nfs
    plan = nfs.Plan(c["n"], c["lags"], c["n_bins"], in_dtype="u16",
                    capacity=max(c["N"], c["lags"][-1] + 1))
    plan.push(frames)
    out = [x.cpu().numpy() for x in plan.structure_function()]
    plan.close()
    return out


def _np(outs):
    return [[x.cpu().numpy() for x in o] for o in outs]


def test_batch_equals_single_plans():
    import paper_1209_3362_amd as nfs
    require_gpu()
    cfgs = _small_batch()
    say("batch: 6 sequences n in {32, 64, 128}, 20..90 u16 frames, 8 lags, 3 streams")
    frames = [gen.make_stack(c, c["seed"], device="cuda") for c in cfgs]
    b = nfs.Batch([_seq(c) for c in cfgs], streams=3)
    got = _np(b.run(frames))
    b.close()
    for c, f, g in zip(cfgs, frames, got):
        want = _single(c, f)
        for x, y in zip(g, want):
            assert np.array_equal(x, y, equal_nan=True), c["name"]


def test_batch_mixed_storage_and_accumulation_equals_single_plans():
    """Sequences of one batch with different spectrum storage and sum
    accumulation (FP32/BF16/FP16, plain/Kahan) each give exactly what a
    single plan with the same options gives."""
    import paper_1209_3362_amd as nfs
    require_gpu()
    cfgs = _small_batch(count=6, seed=11)
    opts = [("f32", "plain"), ("bf16", "kahan"), ("f16", "plain"), ("f32", "kahan"),
            ("bf16", "plain"), ("f16", "kahan")]
    say("batch: 6 sequences with mixed storage/accumulation, 3 streams, seed 11")
    frames = [gen.make_stack(c, c["seed"], device="cuda") for c in cfgs]
    seqs = [dict(_seq(c), spec=sp, accum=ac) for c, (sp, ac) in zip(cfgs, opts)]
    b = nfs.Batch(seqs, streams=3)
    got = _np(b.run(frames))
    b.close()
    for c, f, g, (sp, ac) in zip(cfgs, frames, got, opts):
        plan = nfs.Plan(c["n"], c["lags"], c["n_bins"], in_dtype="u16",
                        capacity=max(c["N"], c["lags"][-1] + 1), spec=sp, accum=ac)
        plan.push(f)
        want = [x.cpu().numpy() for x in plan.structure_function()]
        plan.close()
        for x, y in zip(g, want):
            assert np.array_equal(x, y, equal_nan=True), (c["name"], sp, ac)


def test_batch_graph_replays():
    """Three replays with eager work and a change of the frame data between
    them; every replay equals an eager batch run on the data it read."""
    import paper_1209_3362_amd as nfs
    require_gpu()
    cfgs = _small_batch(count=5, seed=8)
    say("batch graph: 5 sequences, capture once, replay 3 times")
    frames = [gen.make_stack(c, c["seed"], device="cuda") for c in cfgs]
    alt = [gen.make_stack(c, c["seed"] + 100, device="cuda") for c in cfgs]
    b = nfs.Batch([_seq(c) for c in cfgs], streams=4)
    eager = _np(b.run(frames))
    eager_alt = _np(b.run(alt))
    outs = b.capture(frames)
    for rep in range(3):
        src = alt if rep == 1 else frames
        if rep == 1:
            for f, a in zip(frames, alt):
                f.copy_(a)
        if rep == 2:
            for j, (f, c) in enumerate(zip(frames, cfgs)):
                f.copy_(gen.make_stack(c, c["seed"], device="cuda"))
        torch.cuda.synchronize()
        _ = (torch.randn(1000, device="cuda") ** 2).sum().item()  # eager work between
        got = _np(b.replay())
        want = eager_alt if rep == 1 else eager
        for g, w, c in zip(got, want, cfgs):
            for x, y in zip(g, w):
                assert np.array_equal(x, y, equal_nan=True), (rep, c["name"])
        del src
    b.close()


def test_batch_windowed_budget_matches_oracle():
    import paper_1209_3362_amd as nfs
    require_gpu()
    cfgs = gen.batch_workload(master_seed=9, count=4, sizes=(64, 128), frames=(150, 250))
    for c in cfgs:
        c["lags"] = gen.log_spaced_lags(16, 6)
    full = [max(c["N"], c["lags"][-1] + 1) for c in cfgs]
    seqs = [(c["n"], c["lags"], c["n_bins"], "u16", c["N"], "f32") for c in cfgs]
    sizes = [nfs.workspace_size(c["n"], c["lags"], c["n_bins"], capacity=cap)
             for c, cap in zip(cfgs, full)]
    budget = int(0.6 * sum(sizes))
    caps = nfs.batch_capacities(seqs, budget)
    say(f"batch: 4 sequences under a budget of 60% of their whole stacks, rings {caps}")
    assert any(cap < c["N"] for cap, c in zip(caps, cfgs))
    assert all(cap >= min(full_j, c["lags"][-1] + 64) for cap, c, full_j in zip(caps, cfgs, full))
    frames = [gen.make_stack(c, c["seed"], device="cuda") for c in cfgs]
    b = nfs.Batch([_seq(c, cap) for c, cap in zip(cfgs, caps)], streams=2)
    assert b.workspace.numel() <= budget
    got = _np(b.run(frames))
    b.close()
    for c, f, g in zip(cfgs, frames, got):
        ref = oracle.structure_function(f.cpu().numpy().astype(np.float64), c["lags"],
                                        c["n_bins"])
        assert_D_close(g[0], ref["D"], rtol=1e-4)
        assert np.array_equal(g[1], ref["counts"]) and np.array_equal(g[2], ref["pairs"])


def test_batch_orders_after_the_current_stream():
    """Frames still being written on the current stream when the batch is
    run (no synchronisation in between) are read only once complete: the
    batch's streams wait for the current stream, and the current stream
    waits for the batch before the outputs are read."""
    import paper_1209_3362_amd as nfs
    require_gpu()
    cfgs = _small_batch(count=4, seed=12)
    say("batch ordering: 4 sequences, frames drawn and run without a synchronisation")
    b = nfs.Batch([_seq(c) for c in cfgs], streams=3)
    torch.cuda.synchronize()
    frames = [gen.make_stack(c, c["seed"], device="cuda") for c in cfgs]
    # more work on the current stream right before the run, touching the frames
    for f in frames:
        f.copy_(f.flip(0).flip(0))
    got = _np(b.run(frames, sync=False))
    b.close()
    for c, f, g in zip(cfgs, frames, got):
        want = _single(c, f)
        for x, y in zip(g, want):
            assert np.array_equal(x, y, equal_nan=True), c["name"]


@pytest.fixture(scope="module")
def c4_full():
    """The 16-sequence batching workload (n 256..2048, 200..2000 frames, 32
    log-spaced lags to N/2 each, master seed 4) drawn on the GPU once."""
    require_gpu()
    cfgs = gen.batch_workload(master_seed=4)
    say("batch full size: 16 sequences drawn on the GPU (master seed 4)")
    frames = [gen.make_stack(c, c["seed"], device="cuda") for c in cfgs]
    torch.cuda.synchronize()
    return cfgs, frames


@pytest.fixture(scope="module")
def c4_replayed(c4_full):
    """The full workload captured once as a four-stream graph and replayed
    twice, with eager work between the replays; both replays must agree bit
    for bit. Returns the second replay's outputs on the host."""
    import paper_1209_3362_amd as nfs
    cfgs, frames = c4_full
    say("batch full size: capture a four-stream graph, replay twice")
    b = nfs.Batch([_seq(c) for c in cfgs], streams=4)
    b.capture(frames)
    first = _np(b.replay())
    _ = (torch.randn(4096, device="cuda") ** 2).sum().item()
    second = _np(b.replay())
    b.close()
    for x, y, c in zip(first, second, cfgs):
        for u, v in zip(x, y):
            assert np.array_equal(u, v, equal_nan=True), c["name"]
    return second


# every sequence of 2048^2 frames and the longest sequence (1926 frames of 512^2)
C4_ORACLE_SEQS = [1, 4, 5, 15, 9]


@pytest.mark.parametrize("j", C4_ORACLE_SEQS)
def test_batch_workload_graph_replay_matches_oracle(c4_full, c4_replayed, j):
    """Graph replays of the full batching workload against the FP64 oracle
    on sampled rings (six per sequence, from the first to the last ring):
    counts and pairs exact, D within 1e-4."""
    import os
    cfgs, frames = c4_full
    c = cfgs[j]
    nb = c["n_bins"]
    bins = [1, 2, 7, nb // 8, nb // 2 - 1, nb - 1]
    say(f"batch full size vs oracle: {c['name']} (n {c['n']}, {c['N']} frames), rings {bins}")
    host = frames[j].cpu().numpy()
    ref = oracle.structure_function_bins(host, c["lags"], nb, bins,
                                         workers=min(16, os.cpu_count() or 1))
    D, C, P, st = c4_replayed[j]
    assert int(st.reshape(-1)[0]) == 0
    assert np.array_equal(C[bins], ref["counts"]) and np.array_equal(P, ref["pairs"])
    worst = assert_D_close(D[:, bins], ref["D"], rtol=1e-4)
    print(f"{c['name']} replay vs oracle worst relative error {worst:.2e}")


def test_batch_workload_full_size_equals_single_plans(c4_full):
    """The 16-sequence workload the benchmark times (n 256..2048, 200..2000
    frames, 32 lags each), run as one four-stream batch, equals single plans
    on the same frames bit for bit for every sequence."""
    import paper_1209_3362_amd as nfs
    require_gpu()
    cfgs, frames = c4_full
    say("batch full size: eager four-stream run")
    b = nfs.Batch([_seq(c) for c in cfgs], streams=4)
    got = _np(b.run(frames))
    b.close()
    del b
    for c, f, g in zip(cfgs, frames, got):
        say(f"batch full size: single plan for {c['name']} (n {c['n']}, {c['N']} frames)")
        want = _single(c, f)
        for x, y in zip(g, want):
            assert np.array_equal(x, y, equal_nan=True), c["name"]
        assert g[3] == 0
