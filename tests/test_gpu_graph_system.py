"""The registration system after the matching, captured as one HIP graph:
block-based FAST on the sensed image, describe + Fast-NCC, projective
RANSAC and rectification, recorded once on a capture stream and replayed.
Every replay, with eager work and synchronisations between replays, must
reproduce the eager results exactly (the kernels use no memsets and no
floating-point atomics, so the results are deterministic)."""
import numpy as np
import pytest

from paper_2202_13347_amd import sfoc as S
from paper_2202_13347_amd import synth

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def test_system_graph_replays_match_eager():
    assert torch.cuda.is_available()
    S.lib()
    rec = synth.WARP
    w = synth.make_warp_pair(3, rec)
    size, m, r = rec["size"], rec["m"], rec["r"]
    margin = (m + 1) // 2 + r
    dev = torch.device("cuda:0")
    ref = torch.from_numpy(w.ref).to(dev)
    sen = torch.from_numpy(w.sen).to(dev)
    nb = 20
    det = S.Detector(size, size, nb, nb, 1, 0.05, margin, device=dev)
    reg = S.Registrar(size, size, size, size, nb * nb, m, r, S.preset("baseline"), device=dev)
    rs = S.Ransac(nb * nb, S.ransac_params(S.MODEL_PROJECTIVE, 1024, (size, size, size, size), 1.5, 2), device=dev)
    words = torch.from_numpy(synth.ransac_words(3, 1024, 4).view(np.int32)).to(dev)
    rect = torch.empty_like(sen)

    def system(stream):
        ips, _, _, _ = det(sen, stream=stream)
        cps = reg(ref, sen, ips, stream=stream)
        rs(cps, words, stream=stream)
        S.rectify(sen, rs.model, (size, size), fill=0.0, out=rect, stream=stream)

    # eager reference (also sets every kernel's attributes before capture)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        system(s)
    torch.cuda.synchronize()
    want = (det.ips.clone(), reg.cps.clone(), rs.model.clone(), rs.info.clone(), rect.clone())
    assert int(det.n_out.item()) == nb * nb and int(rs.info[3].item()) == 0

    g = torch.cuda.CUDAGraph()
    cap = torch.cuda.Stream()
    with torch.cuda.stream(cap):
        with torch.cuda.graph(g, stream=cap):
            system(cap)
    torch.cuda.synchronize()
    for k in range(3):
        # clobber the outputs eagerly, then replay
        det.ips.fill_(-7)
        reg.cps.fill_(-7)
        rs.model.fill_(0.0)
        rect.fill_(123.0)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        got = (det.ips, reg.cps, rs.model, rs.info, rect)
        for a, b in zip(got, want):
            assert torch.equal(a, b), k
