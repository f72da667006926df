"""Writes the oracle's CP decisions for every interest point of a full-size
workload, for the GPU parity tests and the benchmark's parity report.

    python tests/golden/make_oracle_cps.py scene    # 2048^2, 400 IPs, m 64, r 32
    python tests/golden/make_oracle_cps.py large    # 10000^2, 5000 IPs, m 64, r 48

Only the oracle (oracle/sfoc_oracle.py, through tests/oracle_pool.py) and the
seeded input generator run here.  Every CP is the oracle's
match_one_region: FP64 SFOC of the template and search crops (Section 2.1),
Eq. 9-16 and the peak decision (Section 3.2.2), for three storages of the
descriptor: unrounded (O64) and rounded to bfloat16 / float16 before the
matching (O64q).  The flags are those before the consistency check.

Stored per storage kind k in {o64, bf16, f16}:
  k_rec    n x 5 float64: dy, dx, sub_dy, sub_dx, score
  k_flags  n uint32
  k_ties   K x 3 int32: (cp, dy, dx) of every other offset whose NCC lies
           within 2e-4 * |peak| of the peak (the tie rule of the design
           notes: such a CP has several correct integer answers)
and the sha256 of the inputs (reference, sensed, IPs as stored float32 /
int32 bytes), so a test can tell that it regenerated the same pair.
A 10000^2 run takes about an hour of single-core oracle time, spread over
the host's cores."""
from __future__ import annotations

import hashlib
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

KINDS = (("o64", None), ("bf16", "bf16"), ("f16", "f16"))
TIE_REL = 2e-4


def input_digest(ref, sen, ips) -> str:
    h = hashlib.sha256()
    for a, dt in ((ref, np.float32), (sen, np.float32), (ips, np.int32)):
        h.update(np.ascontiguousarray(a, dt).tobytes())
    return h.hexdigest()


def path_for(name: str) -> str:
    return os.path.join(ROOT, "tests", "golden", f"oracle_cps_{name}.npz")


def workload(name: str):
    from paper_2202_13347_amd import synth
    rec = {"scene": synth.SCENE, "large": synth.LARGE}[name]
    return synth.workload(rec, 0)


def main(name: str):
    from oracle import sfoc_oracle as O
    from tests.oracle_pool import oracle_cps
    t0 = time.time()
    pr, ips, m, r = workload(name)
    print(f"{name}: generated in {time.time() - t0:.1f} s, {len(ips)} IPs", flush=True)
    t0 = time.time()
    res = oracle_cps(pr.ref, pr.sen, ips, m, r, O.Params(), quantise=[q for _, q in KINDS])
    print(f"{name}: oracle in {time.time() - t0:.1f} s", flush=True)
    V = 2 * r + 1
    out = {"digest": np.array(input_digest(pr.ref, pr.sen, ips)), "m": np.int32(m), "r": np.int32(r),
           "shift": np.asarray(pr.shift, np.float64)}
    for (k, _), (rec, surf) in zip(KINDS, res):
        out[k + "_rec"] = np.stack([rec["dy"], rec["dx"], rec["sub_dy"], rec["sub_dx"], rec["score"]], 1) \
            .astype(np.float64)
        out[k + "_flags"] = rec["flags"].astype(np.uint32)
        ties = []
        for i in range(len(rec)):
            if rec["flags"][i] & (O.OOB | O.FLAT_T | O.FLAT_S | O.NONFINITE):
                continue
            s = surf[i].ravel()
            io = (int(rec["dy"][i]) + r) * V + int(rec["dx"][i]) + r
            pk = s[io]
            for j in np.nonzero(s >= pk - TIE_REL * abs(pk))[0]:
                if j != io:
                    ties.append((i, j // V - r, j % V - r))
        out[k + "_ties"] = np.asarray(ties, np.int32).reshape(-1, 3)
        print(f"{name} {k}: {len(out[k + '_ties'])} tie entries, flags {np.bincount(rec['flags'])}", flush=True)
    np.savez_compressed(path_for(name), **out)
    print("wrote", path_for(name))


if __name__ == "__main__":
    main(sys.argv[1] if len(sys.argv) > 1 else "scene")
