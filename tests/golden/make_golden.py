"""Writes tests/golden/oracle_small.json (inputs and oracle outputs for a few
small seeded cases, including ties and one D=6 case) and
tests/golden/diagnostics.json (the oracle's per-workload diagnostics for the
four seeded benchmark workloads).  Calls only oracle/ and the seeded input
generators.

The paper prints no worked numeric example of the likelihood, so these values
are a regression record of the pinned oracle, not published numbers."""
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))
import oracle  # noqa: E402


def cases():
    rng = np.random.default_rng(2010_02994)
    out = []
    for n, d, ties in ((3, 1, 0), (6, 2, 1), (9, 2, 2), (7, 3, 0), (8, 6, 1)):
        x = rng.standard_normal((n, d))
        t = np.sort(rng.uniform(0, 3, n))
        for _ in range(ties):
            i = int(rng.integers(1, n))
            t[i] = t[i - 1]
        t = np.sort(t)
        p = np.array([0.6, 1.1, 1.3, 0.4, 0.9, 0.7])
        out.append((x, t, p))
    return out


def workload_diagnostics():
    from paper_2010_02994_amd import workloads as W
    out = {}
    for name, w in (("c0", W.config0()), ("c1", W.config1(snapshots=0)), ("c2", W.config2()), ("c3", W.config3())):
        d = oracle.diagnostics(w.x, w.t, w.params)
        d["workload"] = w.name
        out[name] = d
    with open(os.path.join(HERE, "diagnostics.json"), "w") as f:
        json.dump({"source": "oracle/oracle.c (oracle_log_rates, oracle_loglik_grad) via tests/golden/make_golden.py",
                   "workloads": out}, f, indent=1)


def main():
    recs = []
    for x, t, p in cases():
        st, ll, gx, gp = oracle.loglik_grad(x, t, p)
        recs.append({"x": x.tolist(), "t": t.tolist(), "params": p.tolist(), "status": st,
                     "loglik": ll, "grad_x": gx.tolist(), "grad_params": gp.tolist()})
    with open(os.path.join(HERE, "oracle_small.json"), "w") as f:
        json.dump({"source": "oracle/oracle.c via tests/golden/make_golden.py",
                   "param_order": ["mu", "h", "tau", "theta", "omega", "xi"], "cases": recs}, f, indent=1)


if __name__ == "__main__":
    main()
    workload_diagnostics()
