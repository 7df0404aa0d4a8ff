"""Parity of the HIP path (through the C ABI) with the FP64 oracle.

Bar: bin indices, bin counts and pair counts bit-exact; exact zeros (lag 0,
the DC-only bin) exactly zero; D within 1e-4 relative of the oracle (FP32
transforms and per-mode FP32 pair sums, FP64 bin sums).
"""
import math

import numpy as np
import pytest
import torch

import gen
import oracle
from gpu_util import assert_D_close, require_gpu, run_plan, say

pytestmark = pytest.mark.gpu


def _half_plane(a, n):
    """Full-plane [n][n] array -> stored half-plane [n][n/2] (k_x = 0..n/2-1)."""
    return np.asarray(a)[:, : n // 2]


def test_c1_parity():
    cfg = gen.config("c1")
    say("c1 parity: 64 frames 128x128 f32, lags 1,2,4,8,16, 64 bins, seed 1")
    f = gen.make_stack(cfg, 1)
    ref = oracle.structure_function(f.numpy(), cfg["lags"], cfg["n_bins"])
    D, C, P, st = run_plan(f, cfg["lags"], cfg["n_bins"], "f32")
    assert st == 0
    assert np.array_equal(C, ref["counts"])
    assert np.array_equal(P, ref["pairs"])
    assert np.all(D[:, 0] == 0.0)  # bin 0 is the DC mode alone
    worst = assert_D_close(D, ref["D"], rtol=1e-4)
    print("c1 worst relative error", worst)


@pytest.mark.parametrize("n,nb", [(16, 8), (16, 1), (128, 64), (128, 7), (1024, 512), (1024, 100)])
def test_bin_map_and_counts_bit_exact(n, nb):
    import paper_1209_3362_amd as nfs
    require_gpu()
    say(f"bin map n={n} nb={nb}")
    plan = nfs.Plan(n, [1], nb, in_dtype="f32", capacity=4)
    got = plan.bin_map().cpu().numpy()
    plan.close()
    want = _half_plane(oracle.bin_index(n, nb), n)
    assert np.array_equal(got, want)
    # counts through the binning kernel
    f = np.ones((3, n, n), dtype=np.float32)
    _, C, _, _ = run_plan(f, [1], nb, "f32")
    assert np.array_equal(C, oracle.bin_counts(oracle.bin_index(n, nb), nb))


def test_spectra_match_oracle():
    import paper_1209_3362_amd as nfs
    require_gpu()
    cfg = gen.config("c1", N=6)
    say("spectra c1 frames, 6 frames")
    f = gen.make_stack(cfg, 3)
    spec = oracle.spectra(oracle.normalise(f.numpy())[0])
    plan = nfs.Plan(128, [1], 64, in_dtype="f32", capacity=6)
    plan.push(f.cuda())
    bidx = _half_plane(oracle.bin_index(128, 64), 128)
    stored = bidx >= 0
    for t in range(6):
        g = plan.spectrum(t).cpu().numpy()
        o = _half_plane(spec[t], 128)
        assert g[0, 0] == 128 * 128
        assert np.all(g[~stored] == 0)
        err = np.abs(g[stored] - o[stored]).max()
        assert err <= 2e-6 * np.abs(o[stored]).max(), err
    plan.close()


def test_power_spectra_match_oracle():
    """nfs_power_spectra_2d against the oracle's per-delay 2D spectra P_tau(k)
    (the paper's differences area): stored modes within 1e-4 relative (plus
    1e-6 of the delay's largest value), other modes 0, tau = 0 exactly 0,
    delays without pairs NaN."""
    import paper_1209_3362_amd as nfs
    require_gpu()
    cfg = gen.config("c1", N=20)
    lags = [0, 1, 3, 7, 19, 20, 25]
    say("power spectra: 20 frames 128x128 f32, lags 0,1,3,7,19,20,25, seed 5")
    f = gen.make_stack(cfg, 5)
    ref = oracle.structure_function(f.numpy(), lags, 64, return_power=True)
    plan = nfs.Plan(128, lags, 64, in_dtype="f32", capacity=32)
    plan.push(f.cuda())
    S = plan.power_spectra().cpu().numpy()
    plan.close()
    assert S.shape == (len(lags), 128, 65)
    stored = _half_plane(oracle.bin_index(128, 64), 128) >= 0
    for i, tau in enumerate(lags):
        if 20 - tau <= 0:
            assert np.all(np.isnan(S[i])), tau
            continue
        g = S[i, :, :64]
        assert np.all(S[i, :, 64] == 0) and np.all(g[~stored] == 0)
        if tau == 0:
            assert np.all(g == 0)
            continue
        o = _half_plane(ref["P"][i], 128)
        err = np.abs(g[stored] - o[stored])
        bound = 1e-4 * np.abs(o[stored]) + 1e-6 * np.abs(o[stored]).max()
        assert np.all(err <= bound), (tau, float((err / np.maximum(o[stored], 1e-30)).max()))


def test_u16_parity():
    cfg = gen.config("c2", n=64, N=40, lags=[1, 2, 3, 5, 8, 13, 21, 34, 39], n_bins=32)
    say("u16 parity: 40 frames 64x64 Poisson, 9 lags, 32 bins, seed 4")
    f = gen.make_stack(cfg, 4)
    ref = oracle.structure_function(f.numpy().astype(np.float64), cfg["lags"], 32)
    D, C, P, st = run_plan(f, cfg["lags"], 32, "u16")
    assert st == 0 and np.array_equal(C, ref["counts"]) and np.array_equal(P, ref["pairs"])
    assert_D_close(D, ref["D"], rtol=1e-4)


def test_window_parity():
    cfg = gen.config("c1", n=64, N=30, lags=[1, 3, 9], n_bins=32)
    say("window parity: 30 frames 64x64 f32, Hann window")
    f = gen.make_stack(cfg, 5)
    w = np.outer(np.hanning(64), np.hanning(64)) + 0.05
    w32 = w.astype(np.float32)
    ref = oracle.structure_function(f.numpy(), cfg["lags"], 32, window=w32.astype(np.float64))
    D, C, P, st = run_plan(f, cfg["lags"], 32, "f32", window=torch.from_numpy(w32))
    assert st == 0
    assert_D_close(D, ref["D"], rtol=1e-4)


def test_ring_wrap_and_push_chunking():
    cfg = gen.config("c1", n=64, N=100, lags=[0, 1, 2, 5, 17, 40], n_bins=32)
    say("ring wrap: 100 frames 64x64, capacity 45 and 100, chunks 1/7/64")
    f = gen.make_stack(cfg, 6)
    ref = oracle.structure_function(f.numpy(), cfg["lags"], 32)
    full = run_plan(f, cfg["lags"], 32, "f32", capacity=100)
    assert_D_close(full[0], ref["D"], rtol=1e-4)
    for cap, chunk in [(45, None), (41, 1), (45, 7), (100, 64), (60, 13)]:
        D, C, P, st = run_plan(f, cfg["lags"], 32, "f32", capacity=cap, chunk=chunk)
        assert st == 0 and np.array_equal(P, ref["pairs"])
        assert_D_close(D, ref["D"], rtol=1e-4)
        assert_D_close(D, full[0], rtol=1e-6)


def test_consecutive_lags_across_windows():
    # Waves whose lags are consecutive integers share a register window of
    # older frames; check it with ring wrap, chunked pushes and early chunks.
    cfg = gen.config("c1", n=32, N=150, n_bins=16)
    lags = list(range(0, 23)) + [30, 31, 32, 33, 47]
    say("consecutive lags 0..22 + 30..33 + 47, 150 frames 32x32, capacity 60, chunks 9")
    f = gen.make_stack(cfg, 12)
    ref = oracle.structure_function(f.numpy(), lags, 16)
    for cap, chunk in [(150, None), (60, 9), (48, 1)]:
        D, C, P, st = run_plan(f, lags, 16, "f32", capacity=cap, chunk=chunk)
        assert np.array_equal(P, ref["pairs"])
        assert_D_close(D, ref["D"], rtol=1e-4)


def test_run_twice_is_bitwise_identical():
    cfg = gen.config("c1")
    say("determinism: c1 twice")
    f = gen.make_stack(cfg, 7)
    a = run_plan(f, cfg["lags"], 64, "f32")
    b = run_plan(f, cfg["lags"], 64, "f32")
    assert np.array_equal(a[0], b[0])


def test_reset_reuses_a_plan_exactly():
    """After nfs_reset the first pair launch stores its sums instead of
    adding them: a reused plan gives bit for bit what a fresh plan gives,
    windowed rings included, and a reset plan read before any push gives
    no pairs (D NaN) with the ring counts unchanged."""
    import paper_1209_3362_amd as nfs
    require_gpu()
    cfg = gen.config("c1", n=64, N=60, n_bins=32)
    lags = [1, 3, 7, 20]
    say("reset: 60 frames 64x64 f32, reuse after reset, capacities 60 and 30, seeds 11/12")
    a = gen.make_stack(cfg, 11).cuda()
    b = gen.make_stack(cfg, 12).cuda()
    for cap in (60, 30):
        fresh = nfs.Plan(64, lags, 32, in_dtype="f32", capacity=cap)
        fresh.push(b)
        want = [x.cpu().numpy() for x in fresh.structure_function()]
        fresh.close()
        plan = nfs.Plan(64, lags, 32, in_dtype="f32", capacity=cap)
        plan.push(a)
        plan.structure_function()
        plan.reset()
        plan.push(b)
        got = [x.cpu().numpy() for x in plan.structure_function()]
        for x, y in zip(got, want):
            assert np.array_equal(x, y, equal_nan=True), cap
        plan.reset()
        D, C, P, st = [x.cpu().numpy() for x in plan.structure_function()]
        assert np.all(np.isnan(D)) and np.all(P == 0) and int(st.reshape(-1)[0]) == 0
        assert np.array_equal(C, want[1])
        plan.close()


def test_edge_lags_and_tiny_stacks():
    cfg = gen.config("c1", n=32, N=9, n_bins=16)
    say("edge lags: lag 0, lags >= N, N = 9 and N = 1")
    f = gen.make_stack(cfg, 8)
    lags = [0, 1, 8, 9, 12]
    ref = oracle.structure_function(f.numpy(), lags, 16)
    D, C, P, st = run_plan(f, lags, 16, "f32", capacity=20)
    assert P.tolist() == [9, 8, 1, 0, 0]
    assert np.all(D[0] == 0.0)
    assert np.all(np.isnan(D[3:]))
    assert_D_close(D, ref["D"], rtol=1e-4)
    D1, _, P1, _ = run_plan(f[:1], [0, 1], 16, "f32", capacity=4)
    assert P1.tolist() == [1, 0] and np.all(D1[0] == 0) and np.all(np.isnan(D1[1]))


def test_degenerate_frame_sets_status():
    say("degenerate frame: an all-zero frame")
    f = np.ones((5, 32, 32), dtype=np.float32)
    f[2] = 0.0
    D, C, P, st = run_plan(f, [1], 16, "f32")
    from paper_1209_3362_amd.nfs import NFS_E_DEGENERATE_FRAME
    assert st == NFS_E_DEGENERATE_FRAME


@pytest.mark.parametrize("n,N", [(16, 12), (32, 10), (256, 8), (512, 6), (1024, 6), (2048, 4),
                                 (4096, 3)])
def test_frame_sizes(n, N):
    cfg = gen.config("c1", n=n, N=N, n_bins=n // 2)
    lags = sorted({1, 2, N - 1})
    say(f"frame size n={n} N={N}")
    f = gen.make_stack(cfg, 9)
    ref = oracle.structure_function(f.numpy(), lags, n // 2)
    D, C, P, st = run_plan(f, lags, n // 2, "f32")
    assert st == 0 and np.array_equal(C, ref["counts"])
    assert_D_close(D, ref["D"], rtol=1e-4)


def test_cosine_closed_form_on_gpu():
    n, N, nb = 64, 40, 32
    modes = [(3, 5, 0.05, 0.37), (-9, 2, 0.02, 1.3), (0, 11, 0.03, 2.0)]
    say("closed form: cosine stack 64x64")
    f = gen.cosine_stack(n, N, modes, dtype=np.float32)
    lags = [1, 2, 5, 11, 23]
    D, C, P, st = run_plan(f, lags, nb, "f32")
    bidx = oracle.bin_index(n, nb)
    want = np.zeros((len(lags), nb))
    for (ky, kx, eps, om) in modes:
        b = bidx[ky % n, kx % n]
        for i, tau in enumerate(lags):
            want[i, b] += (eps * n * n) ** 2 * (1 - math.cos(om * tau)) / C[b]
    hit = want > 0
    # The closed form holds for exact cosines; the frames are rounded to
    # float32 (relative 6e-8 per pixel), which moves D by ~1e-7 relative,
    # and the FP32 transform adds ~1e-7 per stored coefficient: the FP32
    # bar of 1e-5 leaves two orders of margin.
    rel = np.abs(D[hit] / want[hit] - 1)
    print("cosine closed form worst relative error", rel.max())
    assert np.all(rel < 1e-5)
    # off-mode bins hold only FP32 transform leakage
    assert np.all(np.abs(D[~hit]) < 1e-6 * want.max())


@pytest.mark.parametrize("lags", [[1, 100, 545, 600], [3, 900, 1500], [2, 1200, 2400],
                                  gen.log_spaced_lags(700, 32)])
def test_long_lags_use_narrow_tiles(lags):
    """Histories too long for two workgroups per CU: 16 or 8 modes per
    workgroup, one workgroup per CU, up to the largest lag accepted (2400),
    and 32 lags split over eight waves of four."""
    n, N = 32, max(lags) + 60
    cfg = gen.config("c1", n=n, N=N, n_bins=16)
    say(f"long lags {lags}, N={N}, 32x32")
    f = gen.make_stack(cfg, 10)
    ref = oracle.structure_function(f.numpy(), lags, 16)
    D, C, P, st = run_plan(f, lags, 16, "f32")
    assert np.array_equal(P, ref["pairs"])
    assert_D_close(D, ref["D"], rtol=1e-4)


@pytest.mark.parametrize("capacity,accum,chunk", [(4001, "plain", None), (3100, "plain", 333),
                                                  (4001, "kahan", 1000)])
def test_lags_beyond_the_lds_history(capacity, accum, chunk):
    """Delays above 2400 frames (the LDS history's limit) run the
    global-memory pair kernel: with the whole stack resident (delays up to
    one without a pair), with a ring shorter than the stack (sums flushed
    per window) and with Kahan sums."""
    n, N = 16, 4000
    lags = [1, 5, 700, 2401, 3000] + ([3999, 4000] if capacity > 4000 else [])
    cfg = gen.config("c1", n=n, N=N, n_bins=8)
    say(f"lags beyond 2400: {lags}, N={N}, 16x16, ring {capacity}, {accum}, chunk {chunk}")
    f = gen.make_stack(cfg, 12)
    ref = oracle.structure_function(f.numpy(), lags, 8)
    D, C, P, st = run_plan(f, lags, 8, "f32", capacity=capacity, chunk=chunk, accum=accum)
    assert st == 0 and np.array_equal(P, ref["pairs"])
    assert_D_close(D, ref["D"], rtol=1e-4)


def test_short_and_long_lag_groups():
    """99 short delays (two LDS-history launches) and 10 long ones (two
    global-memory launches of 8 and 2) in one plan."""
    n, N = 16, 3000
    lags = list(range(0, 99)) + [2450 + 50 * i for i in range(10)]
    cfg = gen.config("c1", n=n, N=N, n_bins=8)
    say(f"99 short + 10 long lags, N={N}, 16x16")
    f = gen.make_stack(cfg, 13)
    ref = oracle.structure_function(f.numpy(), lags, 8)
    D, C, P, st = run_plan(f, lags, 8, "f32")
    assert np.array_equal(P, ref["pairs"])
    assert_D_close(D, ref["D"], rtol=1e-4)


def test_more_lags_than_one_launch():
    n, N = 32, 260
    lags = list(range(0, 200))
    cfg = gen.config("c1", n=n, N=N, n_bins=16)
    say("200 lags (two lag groups), N=260, 32x32")
    f = gen.make_stack(cfg, 11)
    ref = oracle.structure_function(f.numpy(), lags, 16)
    D, C, P, st = run_plan(f, lags, 16, "f32")
    assert np.array_equal(P, ref["pairs"])
    assert_D_close(D, ref["D"], rtol=1e-4)


def test_bad_calls_raise():
    import paper_1209_3362_amd as nfs
    require_gpu()
    say("argument errors on the device path")
    plan = nfs.Plan(32, [1], 16, in_dtype="u16", capacity=8)
    with pytest.raises(ValueError):
        plan.push(torch.zeros((2, 32, 32), dtype=torch.float32, device="cuda"))
    with pytest.raises(ValueError):
        plan.push(torch.zeros((2, 16, 16), dtype=torch.uint16, device="cuda"))
    with pytest.raises(nfs.NfsError):
        plan.spectrum(0)  # nothing pushed yet
    plan.close()
    with pytest.raises(nfs.NfsError):
        nfs.Plan(32, [1, 1], 16, in_dtype="u16", capacity=8)


def test_tuned_pair_shapes_keep_parity():
    """nfs_tune_pairs times every launch shape on the pushed frames, keeps
    the fastest, and leaves the plan's sums untouched; D afterwards meets
    the oracle."""
    import paper_1209_3362_amd as nfs
    require_gpu()
    cfg = gen.config("c2", n=128, N=300, lags=gen.log_spaced_lags(250, 40), n_bins=64)
    say("tuning: 300 frames 128x128 u16, 40 log-spaced lags to 250, seed 46")
    f = gen.make_stack(cfg, 46)
    ref = oracle.structure_function(f.numpy().astype(np.float64), cfg["lags"], 64)
    plan = nfs.Plan(128, cfg["lags"], 64, in_dtype="u16", capacity=300)
    g = f.cuda()
    plan.push(g[:150])
    shapes = plan.tune_pairs()
    assert shapes and all(m in (16, 8) and 1 <= w <= 12 for m, w in shapes)
    plan.push(g[150:])
    D, C, P, st = plan.structure_function()
    plan.close()
    assert int(st.item()) == 0
    assert np.array_equal(P.cpu().numpy(), ref["pairs"])
    assert_D_close(D.cpu().numpy(), ref["D"], rtol=1e-4)
    print("tuned shapes", shapes)
    plan = nfs.Plan(128, cfg["lags"], 64, in_dtype="u16", capacity=300)
    plan.push(g[:1])
    with pytest.raises(nfs.NfsError) as e:
        plan.tune_pairs()
    assert e.value.status == 7
    plan.close()


@pytest.mark.parametrize("n,N,lags,capacity,chunk", [
    (128, 64, [1, 2, 4, 8, 16], 64, None),             # one window
    (64, 90, [0, 1, 3, 7, 30, 89, 90, 95], 100, 13),   # lag 0, lags without pairs
    (32, 300, list(range(1, 40)), 60, 17),            # ring of 60: many windows
    (16, 3000, [1, 2, 2401, 2600], 2700, 500),        # global-memory kernel
])
def test_work_counters(n, N, lags, capacity, chunk):
    """The library's work counters: frames transformed = N, and the (t, tau)
    pairs the pair kernels summed = sum over lags of max(0, N - tau), each
    counted by the kernels from their own loop decisions."""
    import paper_1209_3362_amd as nfs
    require_gpu()
    cfg = gen.config("c1", n=n, N=N, n_bins=n // 2)
    say(f"work counters: {N} frames {n}x{n}, lags {lags[:6]}..., ring {capacity}, chunk {chunk}")
    f = gen.make_stack(cfg, 14).cuda()
    plan = nfs.Plan(n, lags, n // 2, in_dtype="f32", capacity=capacity)
    for i in range(0, N, chunk or N):
        plan.push(f[i:i + (chunk or N)])
    plan.structure_function()
    frames, pairs = plan.work_counters()
    assert frames == N
    assert pairs == sum(max(0, N - t) for t in lags)
    plan.reset()
    assert plan.work_counters() == (0, 0)
    plan.close()


def test_tuning_cache_and_set_pair_shapes(tmp_path, monkeypatch):
    """The autotuner's choices persist in the JSON cache: a second plan with
    the same key takes them without timing and gives the same D bit for bit;
    nfs_set_pair_shapes refuses shapes the kernel does not support."""
    import paper_1209_3362_amd as nfs
    require_gpu()
    monkeypatch.setenv("NFS_TUNE_CACHE", str(tmp_path / "shapes.json"))
    monkeypatch.delenv("NFS_TUNE_REFRESH", raising=False)
    cfg = gen.config("c2", n=64, N=120, n_bins=32)
    lags = list(range(1, 30)) + [40, 60, 2500]  # two LDS groups? no: one, plus a global one
    say("tuning cache: 120 frames 64x64 u16 (pushed twice over a 2600-slot ring), 32 lags")
    f = gen.make_stack(cfg, 16).cuda()
    out = []
    for k in range(2):
        plan = nfs.Plan(64, lags, 32, in_dtype="u16", capacity=2600)
        plan.push(f)
        shapes = plan.tune_pairs()
        assert plan.tuned_from_cache == (k == 1)
        plan.reset()
        plan.push(f)
        D, _, _, _ = plan.structure_function()
        out.append((shapes, D.cpu().numpy()))
        if k == 1:
            with pytest.raises(nfs.NfsError):
                plan.set_pair_shapes([(16, 99)] + shapes[1:])
            with pytest.raises(nfs.NfsError):
                plan.set_pair_shapes(shapes[:-1])
            assert shapes[-1] == (0, 0)  # the long delay's group
        plan.close()
    assert out[0][0] == out[1][0]
    assert np.array_equal(out[0][1], out[1][1], equal_nan=True)
