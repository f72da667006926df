"""Batched plans on the GPU (through the C ABI): many uneven pairs in one
plan give the per-pair results bit for bit with the default transform
sides, graph replays read fresh image contents, forced and autotuned sides
stay within the oracle tolerances."""
import sys

import numpy as np
import pytest

from oracle import sfoc_oracle as O
from paper_2202_13347_amd import sfoc as S
from paper_2202_13347_amd import synth
from tests.gpu_util import compare_cps, consistency_flip_allowed

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module", autouse=True)
def gpu():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    S.lib()
    yield
    torch.cuda.synchronize()


# seed, (H, W) of the pair, sensed crop (H, W) or None, m, r, n IPs, prior, pitched ref
SPECS = [
    (0, (200, 240), (180, 240), 24, 6, 9, False, False),
    (1, (256, 256), None, 32, 10, 16, True, True),
    (2, (300, 220), (300, 200), 48, 48, 6, False, False),   # 144-px window: one L = 160 transform
    (3, (160, 160), None, 16, 4, 0, False, False),          # no IPs
    (4, (240, 260), None, 32, 20, 12, False, False),
    (5, (220, 220), None, 20, 60, 5, False, True),          # 140-px window (L = 160)
    (6, (340, 330), None, 48, 80, 5, False, False),         # 208-px window: offsets split (2 x 2 blocks, L = 128)
    (7, (300, 300), None, 96, 64, 4, True, False),          # 224-px window: 2 x 2 blocks of L = 160
]
SIDES = (64, 128, 160, 192)


def default_side(m, r):
    return S.match_candidates(m, r)[0]


def build_pairs(specs, seed_shift=0):
    out = []
    for seed, hw, crop, m, r, n, use_prior, pitched in specs:
        pr = synth.make_pair(seed + 100 + seed_shift, hw, max_shift=max(0.0, min(8.0, r - 2.0)))
        sen = pr.sen if crop is None else np.ascontiguousarray(pr.sen[:crop[0], :crop[1]])
        Hs, Ws = sen.shape
        b = (m + 1) // 2 + r
        rng = np.random.default_rng(seed)
        if n:
            ips = synth.random_ips(seed, Hs, Ws, n, b) if min(Hs, Ws) > 2 * b + 1 else np.zeros((0, 2), np.int32)
            ips = np.concatenate([ips, np.array([[2, 3], [Hs - 3, Ws // 2]], np.int32)])   # two out of bounds
        else:
            ips = np.zeros((0, 2), np.int32)
        prior = rng.integers(-3, 4, (len(ips), 2)).astype(np.int32) if use_prior else None
        out.append(dict(ref=pr.ref, sen=sen, ips=ips, prior=prior, m=m, r=r, pitched=pitched, shift=pr.shift))
    return out


def to_device(pairs):
    dp = []
    for q in pairs:
        ref = torch.from_numpy(q["ref"]).cuda()
        if q["pitched"]:
            H, W = ref.shape
            big = torch.full((H, W + 13), float("nan"), device="cuda")
            big[:, :W] = ref
            ref = big[:, :W]
        dp.append(dict(ref=ref, sen=torch.from_numpy(q["sen"]).cuda(), ips=torch.from_numpy(q["ips"]).cuda(),
                       prior=None if q["prior"] is None else torch.from_numpy(q["prior"]).cuda(),
                       m=q["m"], r=q["r"]))
    return dp


def per_pair(dp, p):
    res = []
    for q in dp:
        cps, ncc = S.register_cps(q["ref"], q["sen"], q["ips"], q["m"], q["r"], p, prior=q["prior"],
                                  want_ncc=True)
        res.append((cps.cpu().numpy(), ncc.cpu().numpy()))
    return res


def assert_same(plan, ref_res):
    for k, (c, n) in enumerate(ref_res):
        np.testing.assert_array_equal(plan.cps[k].cpu().numpy(), c, err_msg=f"pair {k}")
        np.testing.assert_array_equal(plan.ncc[k].cpu().numpy(), n, err_msg=f"pair {k}")


@pytest.mark.parametrize("flags", [0, S.PLAN_GRAPH, S.PLAN_DENSE_SEN, S.PLAN_PERSISTENT,
                                   S.PLAN_PERSISTENT | S.PLAN_GRAPH,
                                   # the four-workgroup describe configuration: the same descriptors
                                   S.PLAN_DESCRIBE_ALT, S.PLAN_DESCRIBE_ALT | S.PLAN_GRAPH | S.PLAN_DENSE_SEN])
def test_batched_equals_per_pair(flags):
    say(f"batched vs per-pair, flags {flags}")
    p = S.preset("baseline")
    dp = to_device(build_pairs(SPECS))
    want = per_pair(dp, p)
    plan = S.Plan(dp, p, flags=flags, want_ncc=True)
    info = plan.info()
    assert info["fft_side"] == [default_side(q["m"], q["r"])[0] for q in dp]
    assert info["fft_side"][2] == 160 and info["blocks"][2] == 1
    assert (info["fft_side"][6], info["blocks"][6]) == (128, 2) and (info["fft_side"][7], info["blocks"][7]) == (160, 2)
    for rep in range(2):
        plan()
        torch.cuda.synchronize()
        assert_same(plan, want)
    if flags & S.PLAN_GRAPH:
        assert plan.info()["graph"] == 1
    assert plan.info()["persistent"] == ((1,) * 4 if flags & S.PLAN_PERSISTENT else (0,) * 4)
    assert plan.info()["describe_config"] == (1 if flags & S.PLAN_DESCRIBE_ALT else 0)
    plan.close()


def test_sparse_tiles_count():
    p = S.preset("baseline")
    pairs = build_pairs(SPECS)
    dp = to_device(pairs)
    plan = S.Plan(dp, p)
    want = 0
    for q in pairs:
        Hr, Wr = q["ref"].shape
        Hs, Ws = q["sen"].shape
        want += ((Hr + 31) // 32) * ((Wr + 31) // 32)
        want += len(S.sensed_tiles(q["ips"], q["m"], q["r"], Hs, Ws, Hr, Wr, q["prior"], S.COVER_SMALLER))
    assert plan.info()["describe_tiles"] == want
    plan.close()


def test_graph_replay_reads_new_images():
    say("graph replay with new image contents")
    p = S.preset("baseline")
    dp = to_device(build_pairs(SPECS))
    plan = S.Plan(dp, p, flags=S.PLAN_GRAPH | S.PLAN_DENSE_SEN, want_ncc=True)
    plan()
    torch.cuda.synchronize()
    assert_same(plan, per_pair(dp, p))
    # new contents in the same buffers (and new IP values: dense sensed images)
    new = build_pairs(SPECS, seed_shift=17)
    for q, d in zip(new, dp):
        d["ref"].copy_(torch.from_numpy(q["ref"]))
        d["sen"].copy_(torch.from_numpy(q["sen"]))
        if len(q["ips"]):
            d["ips"].copy_(torch.flip(d["ips"], [0]))
    torch.cuda.synchronize()
    want = per_pair(dp, p)
    for rep in range(3):
        plan()
        torch.cuda.synchronize()
        assert_same(plan, want)
    plan.close()


def oracle_check(q, cps, ncc, p):
    op = O.Params(n_orient=p.n_orient, s1=tuple(p.s1[:p.n_s1]), s2=tuple(p.s2[:p.n_s2]), trunc=p.trunc,
                  sd1=p.sd1, sd2=p.sd2, K=p.K, dil=tuple(p.dil[:p.n_dil]), eps=p.eps)
    o, so = O.register_cps(q["ref"], q["sen"], q["ips"], q["m"], q["r"], op, prior=q["prior"],
                           want_surfaces=True)
    g = S.cps_to_numpy(cps)
    st = compare_cps(g, o, so, q["r"], surf_g=ncc.cpu().numpy(), check_consistency=False)
    allowed = consistency_flip_allowed(o, q["prior"])
    for i in range(len(o)):
        if int(o["flags"][i]) != int(g["flags"][i]):
            assert allowed[i], (i, o[i], g[i])
    return st


@pytest.mark.parametrize("sides", [(64, 128), (128, 64), (160, 192), (192, 160)])
def test_forced_sides_match_oracle(sides):
    # pair 0: 36-px window (default 64); pair 4: 72-px window (default 128, or 64 in two blocks per
    # axis); the 160 and 192 sides with windows narrower than the transform
    say(f"forced transform sides {sides}")
    specs = [SPECS[0], SPECS[4]]
    pairs = build_pairs(specs)
    dp = to_device(pairs)
    for d, L in zip(dp, sides):
        d["fft_side"] = L
    p = S.preset("baseline")
    plan = S.Plan(dp, p, want_ncc=True)
    info = plan.info()
    assert info["fft_side"] == list(sides)
    plan()
    torch.cuda.synchronize()
    for k, q in enumerate(pairs):
        st = oracle_check(q, plan.cps[k], plan.ncc[k], p)
        say(k, sides[k], st)
    plan.close()


def test_autotune_and_cache(tmp_path):
    say("autotune")
    cache = str(tmp_path / "tune.txt")
    p = S.preset("baseline")
    pairs = build_pairs(SPECS)
    dp = to_device(pairs)
    want = per_pair(dp, p)
    plan = S.Plan(dp, p, flags=S.PLAN_AUTOTUNE | S.PLAN_GRAPH, tune_cache=cache, want_ncc=True)
    info = plan.info()
    # every class with IPs and two candidate sides is timed once
    timed = sum(len(S.match_candidates(q["m"], q["r"])) > 1 and len(q["ips"]) > 0 for q in pairs)
    assert timed >= 5
    assert info["tuned_classes"] == timed
    assert info["describe_config"] in (0, 1)   # the faster of the two, timed at creation
    for q, L in zip(pairs, info["fft_side"]):
        assert L in [c[0] for c in S.match_candidates(q["m"], q["r"])]
    plan()
    torch.cuda.synchronize()
    for k, q in enumerate(pairs):
        g = plan.cps[k].cpu().numpy()
        if info["fft_side"][k] == default_side(q["m"], q["r"])[0]:
            np.testing.assert_array_equal(g, want[k][0])
        elif len(q["ips"]):
            oracle_check(q, plan.cps[k], plan.ncc[k], p)
    plan.close()
    plan2 = S.Plan(dp, p, flags=S.PLAN_AUTOTUNE, tune_cache=cache)
    i2 = plan2.info()
    assert i2["tuned_classes"] == 0 and i2["cached_classes"] == timed
    assert i2["fft_side"] == info["fft_side"]
    plan2.close()


def test_corrupt_cache_is_ignored(tmp_path):
    """A cache whose lines name sides the classes cannot use (or do not
    parse) is ignored: every class is timed again and the plan computes
    what per-pair calls compute with the chosen sides."""
    say("autotune with a corrupt cache")
    cache = tmp_path / "tune.txt"
    p = S.preset("baseline")
    pairs = build_pairs(SPECS)
    lines = ["not a cache line", "gfx950/256cu 16 0 1 2"]
    for q in pairs:
        lines.append(f"gfx950/256cu 16 0 {q['m']} {q['r']} 96")     # no such transform side
        lines.append(f"gfx950/256cu 16 0 {q['m']} {q['r']} 128 64")  # trailing field
    cache.write_text("\n".join(lines) + "\n")
    dp = to_device(pairs)
    plan = S.Plan(dp, p, flags=S.PLAN_AUTOTUNE, tune_cache=str(cache), want_ncc=True)
    info = plan.info()
    timed = sum(len(S.match_candidates(q["m"], q["r"])) > 1 and len(q["ips"]) > 0 for q in pairs)
    assert info["cached_classes"] == 0 and info["tuned_classes"] == timed
    for q, L in zip(pairs, info["fft_side"]):
        assert L in [c[0] for c in S.match_candidates(q["m"], q["r"])]
    plan()
    torch.cuda.synchronize()
    for k, q in enumerate(pairs):
        if info["fft_side"][k] == default_side(q["m"], q["r"])[0]:
            continue
        if len(q["ips"]):
            oracle_check(q, plan.cps[k], plan.ncc[k], p)
    plan.close()


@pytest.mark.parametrize("kind", ["bf16", "f16"])
def test_rounded_storage_plan(kind):
    """BF16 / FP16 descriptor storage in a batched plan (graph, sparse
    sensed tiles, split offsets included): bit for bit the per-pair calls
    with the same storage, and the oracle on the same rounded descriptors
    (O64q) for pairs with IPs."""
    say("batched plan with storage", kind)
    p = S.preset("baseline", dtype={"bf16": S.DTYPE_BF16, "f16": S.DTYPE_F16}[kind])
    pairs = build_pairs(SPECS)
    dp = to_device(pairs)
    want = per_pair(dp, p)
    plan = S.Plan(dp, p, flags=S.PLAN_GRAPH, want_ncc=True)
    for rep in range(2):
        plan()
        torch.cuda.synchronize()
        assert_same(plan, want)
    for k in (1, 2, 4):
        q = pairs[k]
        o, so = O.register_cps(q["ref"], q["sen"], q["ips"], q["m"], q["r"], O.Params(), prior=q["prior"],
                               quantise=kind, want_surfaces=True)
        g = S.cps_to_numpy(plan.cps[k])
        st = compare_cps(g, o, so, q["r"], surf_g=plan.ncc[k].cpu().numpy(), check_consistency=False)
        say("  pair", k, st)
    plan.close()


# pairs the direct form takes (2r + 1 <= 32, m <= 64): small and odd m, r = 1, the largest window
# (m 64, r 15: 94 columns, six 16-column chunks), a prior and a pitched reference
DIRECT_SPECS = [
    SPECS[0], SPECS[1], SPECS[3],
    (8, (260, 250), None, 64, 15, 10, True, False),
    (9, (120, 130), None, 5, 1, 8, False, False),
    (10, (200, 200), (150, 170), 33, 7, 11, False, True),
]


@pytest.mark.parametrize("kind", ["bf16", "f16"])
def test_direct_form_matches_oracle(kind):
    """The direct form (R_ST summed in space on the matrix cores) against
    the oracle on the same rounded descriptors, surfaces included, in a
    captured plan replayed twice; the autotuner may pick it for 16-bit
    storage and its choice stays within the oracle's tolerances."""
    say("direct form", kind)
    p = S.preset("baseline", dtype={"bf16": S.DTYPE_BF16, "f16": S.DTYPE_F16}[kind])
    pairs = build_pairs(DIRECT_SPECS)
    dp = to_device(pairs)
    for d in dp:
        d["fft_side"] = S.MATCH_DIRECT
    plan = S.Plan(dp, p, flags=S.PLAN_GRAPH, want_ncc=True)
    info = plan.info()
    assert info["fft_side"] == [S.MATCH_DIRECT] * len(pairs)
    assert info["direct_items"] == sum(len(q["ips"]) for q in pairs)
    assert info["match_items"] == (0, 0, 0, 0)
    first = None
    for rep in range(2):
        plan()
        torch.cuda.synchronize()
        got = [(plan.cps[k].cpu().numpy(), plan.ncc[k].cpu().numpy()) for k in range(len(pairs))]
        if first is None:
            first = got
        else:
            for (c0, n0), (c1, n1) in zip(first, got):
                np.testing.assert_array_equal(c0, c1)
                np.testing.assert_array_equal(n0, n1)
    for k, q in enumerate(pairs):
        if not len(q["ips"]):
            continue
        o, so = O.register_cps(q["ref"], q["sen"], q["ips"], q["m"], q["r"], O.Params(), prior=q["prior"],
                               quantise=kind, want_surfaces=True)
        g = S.cps_to_numpy(plan.cps[k])
        st = compare_cps(g, o, so, q["r"], surf_g=plan.ncc[k].cpu().numpy(), check_consistency=False)
        say("  pair", k, st)
    plan.close()
    # autotuned: the direct form is one of the candidates of every class here
    dp = to_device(pairs)
    tplan = S.Plan(dp, p, flags=S.PLAN_AUTOTUNE, want_ncc=True)
    tinfo = tplan.info()
    for q, L in zip(pairs, tinfo["fft_side"]):
        assert L in [c[0] for c in S.match_candidates(q["m"], q["r"])] + [S.MATCH_DIRECT]
    say("  autotuned forms", tinfo["fft_side"])
    tplan()
    torch.cuda.synchronize()
    for k, q in enumerate(pairs):
        if len(q["ips"]):
            o, so = O.register_cps(q["ref"], q["sen"], q["ips"], q["m"], q["r"], O.Params(), prior=q["prior"],
                                   quantise=kind, want_surfaces=True)
            compare_cps(S.cps_to_numpy(tplan.cps[k]), o, so, q["r"], surf_g=tplan.ncc[k].cpu().numpy(),
                        check_consistency=False)
    tplan.close()
