"""Write the small plan-search dataset the learned-versus-additive GPU test
uses, from chunks collected by ``plansearch collect``:

    python -m paper_1305_1183_amd.data.make_plansearch_subset OUT.npz CHUNK.npz ... \\
        --train 0:70 --eval 150:170

It keeps, for the training scripts, one feature row and the median measured
time per unique kernel, and for the evaluation scripts the measured time of
every sampled candidate plan. The routine table for the additive predictor is
stored beside it (JSON, same directory)."""
from __future__ import annotations

import argparse

import numpy as np

from paper_1305_1183_amd import search as SE


def _range(s):
    a, b = s.split(":")
    return list(range(int(a), int(b)))


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("out")
    ap.add_argument("chunks", nargs="+")
    ap.add_argument("--train", default="0:70")
    ap.add_argument("--eval", default="150:170")
    ap.add_argument("--launch-us", type=float, default=None,
                    help="per-launch term of a plan's time (default: fitted on the training scripts' timings)")
    a = ap.parse_args(argv)
    data = SE.merge([dict(np.load(f, allow_pickle=False)) for f in a.chunks])
    X, y = SE.kernel_training_set(data, _range(a.train))
    launch = a.launch_us if a.launch_us is not None else SE.fit_launch_term(data, _range(a.train))
    ev = [s for s in _range(a.eval) if s in set(int(v) for v in data["script_seed"])]
    m = np.isin(data["cand_seed"], ev)
    np.savez_compressed(a.out, X=X.astype(np.float32), y=y.astype(np.float32),
                        cand_seed=data["cand_seed"][m], cand_idx=data["cand_idx"][m],
                        plan_us=data["plan_us"][m].astype(np.float32), launch_us=np.float32(launch))
    print("train kernels %d, eval scripts %d, eval candidates %d, launch term %.3f us" %
          (len(y), len(ev), int(m.sum()), launch))


if __name__ == "__main__":
    main()
