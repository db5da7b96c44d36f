"""Write the stored expected outputs under tests/golden/.

Inputs come from the seeded generators; expected values come from the CPU
oracle only (oracle/), so the files pin later changes of the oracle and give
the GPU path a fixed target.  Run:  python tests/golden/make_golden.py
"""
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
from paper_1311_0380_amd import synth  # noqa: E402

CASES = {
    # small plain fit (uniform constants, 1-2 hits per layer), first 12 events
    "plainfit_uniform_12ev": dict(gen="cfg1", seed=1, n_events=12),
    # scaled-up plain fit shape (lattice constants, planted tracks), 6 events
    "plainfit_lattice_6ev": dict(gen="cfg2", seed=2, n_events=6),
    # uneven batching shape, 20 events
    "uneven_20ev": dict(gen="cfg3", seed=3, n_events=20),
}


def make(case):
    gen = getattr(synth, case["gen"])
    return gen(seed=case["seed"], n_events=case["n_events"])


def main():
    oracle.build(force=False)
    for name, case in CASES.items():
        batch, consts = make(case)
        rc, out, summ = oracle.fit_batch(batch, consts)
        assert rc == 0
        doc = {
            "source": "CPU oracle (oracle/svt_oracle.c) on seeded generator inputs; "
                      "fit of paper Sec. 2 over all combinations, chi2 cut, best per road",
            "inputs": case,
            "summary": {k: int(v) for k, v in summ.items()},
            "results": {k: (v.astype(int).tolist() if k != "chi2" else [int(x) for x in v])
                        for k, v in out.items() if v is not None},
        }
        with open(os.path.join(HERE, name + ".json"), "w") as f:
            json.dump(doc, f, separators=(",", ":"))
        print(name, batch.n_roads, "roads", summ)


if __name__ == "__main__":
    main()
