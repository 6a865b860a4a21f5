"""Writes c1_error_policy.json: the oracle's decisions and metrics for the
error-threshold refresh (eq. error-refresh-rule) on a mixed stream in the
regime of the 100000 x 2000, k = 64 workload, scaled down so that the
oracle's exact ratio (a full SVD of A_t at every check) stays affordable:
6000 x 400, 20 factors, k = 32 (the cut inside the noise bulk, so the
refresh block b = k + k / 2 < n), 600 i.i.d. 80/10/10 row / column / entry
ticks, checks every 50 ticks, gamma chosen so that the policy fires a few
times.  Calls only oracle/ (and synth for the inputs)."""
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from synth import FactorStream, event_schedule_iid          # noqa: E402
from oracle.engine import OracleEngine                     # noqa: E402
from oracle.policies import Policy                         # noqa: E402

PARAMS = {"seed": 93, "m0": 6000, "n0": 400, "K": 20, "k": 32, "T": 600, "mix": [0.8, 0.1, 0.1],
          "gamma": 1.00011, "check_every": 50}


def main():
    p = PARAMS
    fs = FactorStream(seed=p["seed"], stream=0, n0=p["n0"], K=p["K"])
    A0 = fs.initial(p["m0"])
    events = fs.materialize(event_schedule_iid(p["seed"], 0, p["T"], mix=tuple(p["mix"])), m0=p["m0"])
    o = OracleEngine(A0, p["k"], policy=Policy.error(gamma=p["gamma"], check_every=p["check_every"]), cgs2=True)
    checks = []
    for ev in events:
        o.apply(ev)
        if ev.t % p["check_every"] == 0 and ev.t - o.t_last >= p["check_every"]:
            checks.append([ev.t, o.exact_metrics()["frob_ratio"]])
        if o.decide(ev.kind):
            o.refresh(store_reference=True)
            o.refresh_ticks.append(o.t)
        print(ev.t, file=sys.stderr) if ev.t % 100 == 0 else None
    x = o.exact_metrics()
    out = {"params": p, "refresh_ticks": o.refresh_ticks, "checks": checks,
           "final": {"sigma": [float(v) for v in o.s], "frob_error": x["frob_error"], "frob_opt": x["frob_opt"],
                     "m": int(o.A.shape[0]), "n": int(o.A.shape[1])}}
    with open(os.path.join(HERE, "c1_error_policy.json"), "w") as f:
        json.dump(out, f, indent=1)
    print(out["refresh_ticks"], min(abs(r - p["gamma"]) for _, r in checks))


if __name__ == "__main__":
    main()
