"""Host logic of the benchmark: the HBM-traffic lookup in the committed
counter summary (scaled FETCH/WRITE, only while the kernel source is the one
measured) and the algorithmic work counts the roofline divides by."""
import hashlib
import os

import pytest

import bench
from paper_2202_13347_amd import sfoc as S


def _write(path, kernel, sha, fetch=100.0, write=50.0, fs=2.0, ws=1.0):
    path.write_text(f"# header\n\n    traffic {kernel} fetch_kib={fetch} write_kib={write} fetch_scale={fs} "
                    f"write_scale={ws} source=x sha256={sha}\n")


def _sha(kernel):
    src = os.path.join(bench.ROOT, "paper_2202_13347_amd", "csrc", bench.KERNEL_SOURCES[kernel])
    return hashlib.sha256(open(src, "rb").read()).hexdigest()


def test_traffic_scaled_when_source_matches(tmp_path, monkeypatch):
    f = tmp_path / "t.md"
    _write(f, "match", _sha("match"), fetch=100.0, write=50.0, fs=2.0, ws=1.0)
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(f))
    assert bench.stored_traffic("match") == pytest.approx(1024.0 * (100.0 * 2.0 + 50.0 * 1.0))


def test_traffic_none_for_other_source_or_missing_line(tmp_path, monkeypatch):
    f = tmp_path / "t.md"
    _write(f, "match", "0" * 64)
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(f))
    assert bench.stored_traffic("match") is None          # measured on another kernel source
    assert bench.stored_traffic("describe") is None       # no line for this kernel
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(tmp_path / "absent.md"))
    assert bench.stored_traffic("match") is None


def test_committed_summary_parses():
    # every traffic line of the committed summary has the fields the lookup reads
    n = 0
    for line in open(bench.TRAFFIC_FILE):
        f = line.strip().split()
        if f[:1] == ["traffic"]:
            kv = dict(x.split("=", 1) for x in f[2:] if "=" in x)
            assert f[1] in bench.KERNEL_SOURCES
            for k in ("fetch_kib", "write_kib", "fetch_scale", "write_scale", "sha256"):
                assert k in kv
            assert 1.5 < float(kv["fetch_scale"]) < 2.5 and 0.5 < float(kv["write_scale"]) < 1.5
            n += 1
    assert n == len(bench.KERNEL_SOURCES)


def test_work_counts():
    p = S.preset("baseline")
    base = bench.sfoc_flops_per_px(p)
    assert base == 1252.0
    # the first-order-only ablation drops the second-order passes, steering and channels
    q = p.copy()
    q.second_order = 0
    assert bench.sfoc_flops_per_px(q) < base
    # more orientations add steering, smoothing and normalisation work, not convolution work
    r = p.copy()
    r.n_orient = 12
    assert bench.sfoc_flops_per_px(r) > base
    # Fast-NCC: 2z + 1 real 2-D FFTs of side M plus the spectrum products
    assert bench.fastncc_flops_per_ip(128, 16) == 19988480.0
    # linear in the channel count (one shared inverse), quadratic-log in the side
    f = bench.fastncc_flops_per_ip
    assert f(128, 48) - f(128, 32) == f(128, 32) - f(128, 16)
    assert f(128, 16) < 2 * f(128, 8)
    assert 4 * f(64, 16) < f(128, 16) < 5 * f(64, 16)
