"""Oracle CPs for every interest point of a full-size workload, computed in
parallel on the host cores (test infrastructure).

Each CP is the oracle's match_one_region (SFOC of the template and search
crops with their reflect-101 halos, then Eq. 9-16 and the peak decision);
CPs are independent, so they are spread over a pool of worker processes.
The workers are started with the "spawn" method: they are fresh
interpreters that never inherit the parent's GPU handles, and each receives
the two images once, through the pool initializer."""
from __future__ import annotations

import multiprocessing as mp
import os

import numpy as np

_REF = _SEN = _IPS = _ARGS = None


def pool_workers(cap: int = 16) -> int:
    """Worker processes: the host's cores, at most `cap` (16 is the CPU share
    of one GPU on the GPU hosts)."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(cap, n))


def _init(ref, sen, ips, args):
    global _REF, _SEN, _IPS, _ARGS
    os.environ.setdefault("OMP_NUM_THREADS", "1")
    _REF, _SEN, _IPS, _ARGS = ref, sen, ips, args


def _one(k):
    from oracle import sfoc_oracle as O
    m, r, p, prior, quantise = _ARGS
    pr = None if prior is None else prior[k]
    res = O.match_one_region_variants(_REF, _SEN, _IPS[k], m, r, p, prior=pr, quantise=quantise)
    return k, [(rec, np.asarray(s, np.float64)) for rec, s in res]


def oracle_cps(ref, sen, ips, m, r, p, prior=None, quantise=(None,), workers=None, keep_surfaces=True,
               chunks=4):
    """Oracle records (structured, CP_DTYPE, flags before the consistency
    check) and surfaces for every IP, one entry per rounding in `quantise`.
    Returns [(records, surfaces or None)] in the order of `quantise`."""
    from oracle import sfoc_oracle as O
    ips = np.ascontiguousarray(ips, np.int32)
    n = len(ips)
    V = 2 * r + 1
    out = []
    for _ in quantise:
        rec = np.zeros(n, dtype=O.CP_DTYPE)
        rec["sen_row"], rec["sen_col"] = ips[:, 0], ips[:, 1]
        out.append([rec, np.zeros((n, V, V)) if keep_surfaces else None])
    w = workers or pool_workers()
    ctx = mp.get_context("spawn")
    args = (m, r, p, prior, tuple(quantise))
    with ctx.Pool(w, initializer=_init, initargs=(np.asarray(ref), np.asarray(sen), ips, args)) as pool:
        for k, res in pool.imap_unordered(_one, range(n), chunksize=max(1, n // (w * chunks))):
            for j, (rec, s) in enumerate(res):
                R = out[j][0]
                R["dy"][k], R["dx"][k], R["sub_dy"][k], R["sub_dx"][k], R["score"][k], R["flags"][k] = rec
                if keep_surfaces:
                    out[j][1][k] = s
    return [tuple(x) for x in out]
