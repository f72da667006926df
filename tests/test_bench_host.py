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
    # 674 FMA per pixel: 312 convolution + 40 steering + 288 smoothing + 34 normalisation
    assert bench.sfoc_fma_per_px(p) == 674.0
    base = bench.sfoc_flops_per_px(p)
    assert base == 1348.0
    assert bench.sfoc_bytes_per_px(4, 16) == 68.0 and bench.sfoc_bytes_per_px(2, 16) == 36.0
    # the first-order-only ablation drops the second-order passes, steering and channels
    q = p.copy()
    q.second_order = 0
    assert bench.sfoc_flops_per_px(q) < base
    # more orientations add steering, smoothing and normalisation work, not convolution work
    r = p.copy()
    r.n_orient = 12
    assert bench.sfoc_flops_per_px(r) > base
    # Fast-NCC: 2z + 1 real 2-D FFTs of side M, the spectrum products and the
    # NCC assembly: 20.07 Mflop for m 64, r 32 (M 128, V 65)
    f = bench.fastncc_flops_per_ip
    assert f(128, 16, 65) == 19988480.0 + 20.0 * 65 * 65
    assert round(f(128, 16, 65) / 1e6, 1) == 20.1
    assert round(f(160, 16, 97) / 1e6, 1) == 32.8
    # linear in the channel count (one shared inverse), quadratic-log in the side
    assert f(128, 48, 65) - f(128, 32, 65) == f(128, 32, 65) - f(128, 16, 65)
    assert f(128, 16, 65) < 2 * f(128, 8, 65)
    assert 4 * f(64, 16, 33) < f(128, 16, 65) < 5 * f(64, 16, 33)
    # 655 KB per IP at bfloat16 for the scene's windows
    assert bench.fastncc_bytes_per_ip(64, 128, 16, 2) == 16 * 2 * (64 * 64 + 128 * 128)


def test_roof_entry():
    e = bench.roof_entry("x", 1.0, 157.3e9, 1e9)
    assert e["frac_valu_peak"] == pytest.approx(1.0)
    assert e["binding_roof"] == "valu" and e["frac_binding_roof"] == pytest.approx(1.0)
    e = bench.roof_entry("x", 1.0, 1e9, 8e9)         # intensity 1/8 flop per byte: HBM binds
    assert e["binding_roof"] == "hbm" and e["frac_binding_roof"] == pytest.approx(1.0)
    e = bench.roof_entry("x", 2.0, 0.0, 8e9)
    assert e["binding_roof"] == "hbm" and e["frac_hbm_peak"] == pytest.approx(0.5)
    assert bench.roof_entry("x", 0.0, 1.0, 1.0) is None
