"""Host-only planner code (parameter checks, constant synthesis, match plans,
sensed-tile cover and the autotuner cache) compiled with g++ under
AddressSanitizer and UndefinedBehaviorSanitizer, driven by a small C++
program on the CPU.  Nothing here touches a GPU: the planner has no HIP
types, so it builds with the host compiler alone.

The autotuner cache is the one path that reads a file the user may have
edited: a corrupt line must never hand the match launches a transform side
the class cannot use (a side of 64 for a template of 96 would otherwise be
launched with zero offsets per block)."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2202_13347_amd", "csrc")

DRIVER = r'''
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#include <random>
#include "sfoc_plan.h"
using namespace sfoc;

static void show_plan(int m, int r) {
    const MatchPlan p = match_plan(7, m, r);
    int Ls[kNumSides];
    const int n = match_candidates(m, r, Ls);
    printf("plan %d %d %d %d %d %zu cand", m, r, p.L, p.nb, p.Vb, p.ws_bytes);
    for (int k = 0; k < n; ++k) printf(" %d", Ls[k]);
    printf("\n");
}

int main(int argc, char** argv) {
    const char* dir = argv[1];
    char path[1024], out[1024];
    snprintf(path, sizeof path, "%s/cache.txt", dir);
    snprintf(out, sizeof out, "%s/cache_out.txt", dir);
    // ---- cache: read a corrupt file, look up, write, read back ----
    TuneCache c = tune_cache_read(path);
    printf("entries %zu\n", c.size());
    for (const auto& kv : c)
        printf("entry %s %d %d %d %d %d\n", std::get<0>(kv.first).c_str(), std::get<1>(kv.first),
               std::get<2>(kv.first), std::get<3>(kv.first), std::get<4>(kv.first), kv.second);
    const int q[][4] = {{16, 0, 96, 64}, {16, 0, 64, 32}, {16, 0, 48, 16}, {16, 1, 64, 32}, {16, 0, 32, 10},
                        {16, 0, 96, 16}, {12, 0, 64, 32}, {16, 2, 24, 6}, {16, 0, 24, 6}, {16, 1, 48, 16}};
    for (const auto& k : q)
        printf("lookup %d %d %d %d %d\n", k[0], k[1], k[2], k[3], tune_cache_lookup(c, "gfx950/256cu", k[0], k[1], k[2], k[3]));
    // a hand-inserted entry that is not a candidate is refused at lookup too
    c[TuneKey("gfx950/256cu", 16, 0, 96, 64)] = 64;
    printf("lookup_inserted %d\n", tune_cache_lookup(c, "gfx950/256cu", 16, 0, 96, 64));
    c.erase(TuneKey("gfx950/256cu", 16, 0, 96, 64));
    printf("write %d\n", (int)tune_cache_write(out, c));
    const TuneCache back = tune_cache_read(out);
    printf("roundtrip %d\n", (int)(back == c));
    printf("missing %zu\n", tune_cache_read("/nonexistent/dir/cache.txt").size());
    printf("null %zu\n", tune_cache_read(nullptr).size());
    printf("write_null %d\n", (int)tune_cache_write(nullptr, c));
    // ---- params and constants ----
    for (int which = 0; which < 2; ++which) {
        sfoc_params p;
        memset(&p, 0, sizeof p);
        p.trunc = 3.0; p.K = 1; p.n_dil = 3; p.dil[0] = 1; p.dil[1] = 2; p.dil[2] = 3;
        p.sd1 = 1.0; p.sd2 = 1.5; p.eps = 1e-8; p.second_order = 1;
        if (which == 0) { p.n_orient = 6; p.n_s1 = 3; p.s1[0] = 0.6; p.s1[1] = 0.8; p.s1[2] = 1.0; p.n_s2 = 1; p.s2[0] = 1.5; }
        else { p.n_orient = 8; p.n_s1 = p.n_s2 = 3; for (int i = 0; i < 3; ++i) p.s1[i] = p.s2[i] = i + 1; }
        int32_t z = 0;
        const int rc = check_params(&p, &z);
        DescribeConsts dc;
        build_describe_consts(&p, &dc);
        printf("params %d %d %d nsig %d R %d Q %d\n", which, rc, z, dc.nsig, dc.R, dc.Q);
        p.s1[0] = 9.0;                      // radius 27 > 24
        printf("params_big %d\n", check_params(&p, nullptr));
        p.s1[0] = 1.0; p.n_orient = 5;      // z = 10 is not a supported channel count
        printf("params_z %d\n", check_params(&p, nullptr));
    }
    printf("params_null %d\n", check_params(nullptr, nullptr));
    // ---- match plans ----
    const int mr[][2] = {{32, 10}, {64, 32}, {64, 48}, {96, 64}, {48, 16}, {3, 1}, {126, 200}, {127, 1},
                         {2, 5}, {30, 511}, {30, 512}, {1 << 30, 1 << 30}, {2000000000, 5}};
    for (const auto& k : mr) show_plan(k[0], k[1]);
    // ---- sensed tiles: random IPs, some far outside ----
    std::mt19937 rng(7);
    for (int t = 0; t < 200; ++t) {
        const int64_t Hs = 1 + rng() % 300, Ws = 1 + rng() % 300, Hr = 1 + rng() % 300, Wr = 1 + rng() % 300;
        const int m = 3 + rng() % 60, r = 1 + rng() % 40, n = rng() % 50;
        int32_t* ips = (int32_t*)malloc(sizeof(int32_t) * 2 * (n + 1));
        int32_t* pri = (int32_t*)malloc(sizeof(int32_t) * 2 * (n + 1));
        for (int i = 0; i < 2 * n; ++i) {
            ips[i] = (int32_t)(rng() % 700) - 200;
            pri[i] = (int32_t)(rng() % 200) - 100;
        }
        std::vector<std::pair<int, int>> tiles;
        const int cover = t % 3, k = template_tile_rows(m, 32);
        sensed_tiles(ips, (t & 1) ? pri : nullptr, n, m, r, Hs, Ws, Hr, Wr, 32, cover, tiles);
        if ((int64_t)tiles.size() > (int64_t)n * (k + 1) * (k + 1)) printf("too many tiles\n");
        for (const auto& o : tiles)
            if (o.first < 0 || o.first >= Hs || o.second < 0 || o.second >= Ws ||
                (cover == kCoverGrid && (o.first % 32 || o.second % 32)))
                printf("bad tile\n");
        std::vector<uint8_t> wm((size_t)(((Hr + 31) / 32) * ((Wr + 31) / 32)));
        window_tile_mask(ips, (t & 1) ? pri : nullptr, n, m, r, Hs, Ws, Hr, Wr, 32, wm.data());
        free(ips);
        free(pri);
    }
    printf("tiles ok\n");
    printf("ws %zu\n", describe_ws_bytes(2048, 2048));
    return 0;
}
'''

CACHE = """gfx950/256cu 16 0 64 32 128
gfx950/256cu 16 0 48 16 64
gfx950/256cu 16 0 96 64 64
gfx950/256cu 16 0 96 16 128 extra
gfx950/256cu 16 0 96 16 96
gfx950/256cu 16 9 64 32 128
gfx950/256cu -3 0 64 32 128
gfx950/256cu 16 0 32 10
garbage line with words
gfx950/256cu 16 0 32 10 999999999999999999999999
gfx950/256cu 16 1 64 32 128

gfx950/256cu 16 0 2 1 64
gfx950/256cu 16 0 1000000000 1000000000 128
gfx950/256cu 16 0 -1073741824 1073741824 128
gfx950/256cu 16 0 32 10 64
gfx950/256cu 16 2 24 6 1
gfx950/256cu 16 0 24 6 1
gfx950/256cu 16 1 48 16 1
"""


def _build(tmp_path, sanitize):
    exe = tmp_path / "plan_host"
    drv = tmp_path / "driver.cpp"
    drv.write_text(DRIVER)
    flags = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer"] \
        if sanitize else []
    subprocess.run(["g++", "-std=c++17", "-O1", "-g", *flags, "-I", os.path.join(ROOT, "include"), "-I", CSRC,
                    str(drv), os.path.join(CSRC, "sfoc_plan.cpp"), "-o", str(exe)], check=True)
    return exe


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
@pytest.mark.parametrize("sanitize", [True, False])
def test_planner_host_code(tmp_path, sanitize):
    exe = _build(tmp_path, sanitize)
    (tmp_path / "cache.txt").write_text(CACHE)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    env.pop("LD_PRELOAD", None)
    res = subprocess.run([str(exe), str(tmp_path)], capture_output=True, text=True, env=env)
    assert res.returncode == 0, res.stderr
    assert "runtime error" not in res.stderr and "AddressSanitizer" not in res.stderr, res.stderr
    lines = res.stdout.splitlines()
    got = {}
    for l in lines:
        f = l.split()
        got.setdefault(f[0], []).append(f[1:])
    # only the lines that parse completely, with a known dtype, z >= 1 and a
    # form that plan_candidates offers (the direct form: 16-bit dtypes, 2r + 1 <= 32), survive
    entries = sorted(tuple(e) for e in got["entry"])
    assert entries == sorted([("gfx950/256cu", "16", "0", "64", "32", "128"),
                              ("gfx950/256cu", "16", "0", "48", "16", "64"),
                              ("gfx950/256cu", "16", "1", "64", "32", "128"),
                              ("gfx950/256cu", "16", "0", "32", "10", "64"),
                              ("gfx950/256cu", "16", "2", "24", "6", "1")]), entries
    look = {tuple(map(int, e[:4])): int(e[4]) for e in got["lookup"]}
    assert look[(16, 0, 96, 64)] == 0       # the corrupt L = 64 line for m 96 was dropped
    assert look[(16, 0, 64, 32)] == 128
    assert look[(16, 0, 48, 16)] == 64
    assert look[(16, 1, 64, 32)] == 128
    assert look[(16, 0, 32, 10)] == 64
    assert look[(16, 0, 96, 16)] == 0       # a trailing token and a side of 96: both dropped
    assert look[(12, 0, 64, 32)] == 0
    assert look[(16, 2, 24, 6)] == 1        # the direct form, for 16-bit storage only
    assert look[(16, 0, 24, 6)] == 0 and look[(16, 1, 48, 16)] == 0
    assert got["lookup_inserted"] == [["0"]]
    assert got["write"] == [["1"]] and got["roundtrip"] == [["1"]]
    assert got["missing"] == [["0"]] and got["null"] == [["0"]] and got["write_null"] == [["0"]]
    # presets: paper z = 12, baseline z = 16; radius and channel-count limits
    params = {e[0]: e for e in got["params"]}
    assert params["0"][1:3] == ["0", "12"] and params["1"][1:3] == ["0", "16"]
    assert all(e == ["-2"] for e in got["params_big"])
    assert all(e == ["-2"] for e in got["params_z"])
    assert got["params_null"] == [["-1"]]
    plans = {(int(e[0]), int(e[1])): e[2:] for e in got["plan"]}
    assert plans[(64, 32)][:3] == ["128", "1", "65"]
    assert plans[(96, 64)][:3] == ["160", "2", "65"] and plans[(96, 64)][4:] == ["cand", "160", "128", "192"]
    assert plans[(64, 48)][:3] == ["160", "1", "97"]
    assert plans[(2, 5)][0] == "0" and plans[(127, 1)][0] == "160" and plans[(30, 512)][0] == "0"
    assert plans[(1 << 30, 1 << 30)][0] == "0" and plans[(2000000000, 5)][0] == "0"
    assert got["tiles"] == [["ok"]]
    assert "too" not in got and "bad" not in got
