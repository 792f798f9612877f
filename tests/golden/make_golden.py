"""Write the stored expected values under tests/golden/ (calls only oracle/ and synth/).

    python tests/golden/make_golden.py c1_auc    # seconds
    python tests/golden/make_golden.py c2_auc    # about 35 minutes, single thread
    python tests/golden/make_golden.py batch6_auc  # about a minute
    python tests/golden/make_golden.py batch6_bf16_auc  # about five minutes (bfloat16 storage, 8 streams)
    python tests/golden/make_golden.py mid_auc     # about a minute
    python tests/golden/make_golden.py c2_walk_auc   # C2 with random-walk pairs: about 40 minutes
    python tests/golden/make_golden.py mid_walk_auc  # the mid-size graph with random-walk pairs
    python tests/golden/make_golden.py sbm_f1        # labelled graph, node-classification F1: about 10 minutes
    python tests/golden/make_golden.py c2_pool_auc   # C2 with pairs from a pair pool: about 40 minutes
    python tests/golden/make_golden.py sbm_pool_f1   # labelled graph, pair-pool F1: about 5 minutes

Each output JSON records the command, the workload and the oracle's binary64 result.
"""
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import numpy as np  # noqa: E402

import oracle  # noqa: E402
from synth import CONFIGS, config_graph, mid_graph, small_batch  # noqa: E402


# Random-walk pair source of the walk workloads: walk length, window, walks per batch.
WALK = dict(L=100, W=2, Bw=1024)


def run_auc(name: str, orders: int, T: int, d: int, out: str, walks: bool = False, pool: bool = False):
    cfg = CONFIGS[name]
    t0 = time.time()
    g, hs, hd, neg = config_graph(name, holdout=True)
    tb = oracle.Tables(g.n, g.src, g.dst, g.w)
    m = oracle.Model(tb, d=d, K=cfg["K"], orders=orders, T=T, seed=cfg["seed"],
                     eta0=cfg["eta0"])
    wg = oracle.WalkGraph(tb, **WALK) if (walks or pool) else None
    R = oracle.pool_size(T) if pool else 0
    res = {"workload": name, "n": g.n, "m_train": g.m, "held_out": int(hs.size), "d": d,
           "K": cfg["K"], "orders": orders, "T": T, "seed": cfg["seed"], "eta0": cfg["eta0"],
           "mode": "seq", "precision": "binary64",
           "pairs": (f"pair pool of {R} pairs collected from random walks {WALK}" if pool else
                     f"random walks {WALK}" if walks else "arc draws"),
           "command": f"python tests/golden/make_golden.py {sys.argv[1]}"}
    def aucs(prefix):
        """Held-out AUC under each score: order 2 vertex.context (uc) and
        vertex.vertex (uu), order 1 (o1), and the concatenated embedding (concat)."""
        sc = {}
        if orders & 2:
            sc["uc"] = (m.scores(hs, hd, 2), m.scores(hs, neg, 2))
            sc["uu"] = (oracle.pair_scores(m.U, m.U, hs, hd), oracle.pair_scores(m.U, m.U, hs, neg))
        if orders & 1:
            sc["o1"] = (m.scores(hs, hd, 1), m.scores(hs, neg, 1))
        if orders == 3:
            sc["concat"] = (sc["uu"][0] + sc["o1"][0], sc["uu"][1] + sc["o1"][1])
        for k, (p, q) in sc.items():
            res[f"{prefix}auc_{k}"] = oracle.auc(p, q)

    aucs("init_")
    m.train(0, T, "seq", walks=wg, pool=R)
    aucs("")
    res["oracle_seconds"] = round(time.time() - t0, 1)
    with open(os.path.join(HERE, out), "w") as f:
        json.dump(res, f, indent=1)
    print(json.dumps(res))


def run_batch6(out: str, storage: str = "binary64"):
    """Second-order held-out AUCs (uc, uu) of the six small graphs of the batched-launch
    tests, each trained alone in SEQ mode with its own seed and graph id; binary64 tables,
    or bfloat16 tables with every write stochastically rounded (storage="bf16")."""
    t0 = time.time()
    res = {"graphs": [], "K": 5, "orders": 2, "mode": "seq",
           "precision": "binary64" if storage == "binary64" else
           "binary64 arithmetic, bfloat16 tables (nearest-rounded initial values, stochastically rounded writes)",
           "command": f"python tests/golden/make_golden.py {sys.argv[1]}"}
    streams = 1 if storage == "binary64" else 8
    if streams > 1:
        res["rounding_streams"] = streams
        res["note"] = ("auc_uc / auc_uu: mean over the independent rounding streams 0..7; "
                       "sd_*: their sample standard deviation")
    for it in small_batch(6):
        g, hs, hd, neg = it["graph"], it["held_src"], it["held_dst"], it["neg_dst"]
        tb = oracle.Tables(g.n, g.src, g.dst, g.w)
        uc, uu = [], []
        for stream in range(streams):
            m = oracle.Model(tb, d=it["d"], K=5, orders=2, T=it["T"], seed=it["seed"],
                             graph_id=it["graph_id"], storage=storage, sr_stream=stream)
            m.train(0, it["T"], "seq")
            uc.append(oracle.auc(m.scores(hs, hd, 2), m.scores(hs, neg, 2)))
            uu.append(oracle.auc(oracle.pair_scores(m.U, m.U, hs, hd), oracle.pair_scores(m.U, m.U, hs, neg)))
        rec = {"graph_id": it["graph_id"], "n": g.n, "m_train": g.m, "held_out": int(hs.size), "d": it["d"],
               "T": it["T"], "seed": it["seed"], "auc_uc": float(np.mean(uc)), "auc_uu": float(np.mean(uu))}
        if streams > 1:
            rec.update(sd_uc=float(np.std(uc, ddof=1)), sd_uu=float(np.std(uu, ddof=1)), streams_uc=uc,
                       streams_uu=uu)
        res["graphs"].append(rec)
        print(res["graphs"][-1], flush=True)
    res["oracle_seconds"] = round(time.time() - t0, 1)
    with open(os.path.join(HERE, out), "w") as f:
        json.dump(res, f, indent=1)


def run_mid(out: str, walks: bool = False):
    """Second-order held-out AUCs (uc, uu) of the mid-size workload, SEQ mode."""
    t0 = time.time()
    it = mid_graph()
    g, hs, hd, neg = it["graph"], it["held_src"], it["held_dst"], it["neg_dst"]
    tb = oracle.Tables(g.n, g.src, g.dst, g.w)
    m = oracle.Model(tb, d=it["d"], K=5, orders=2, T=it["T"], seed=it["seed"], graph_id=it["graph_id"])
    m.train(0, it["T"], "seq", walks=oracle.WalkGraph(tb, **WALK) if walks else None)
    res = {"workload": "synth.mid_graph", "n": g.n, "m_train": g.m, "held_out": int(hs.size), "d": it["d"],
           "K": 5, "orders": 2, "T": it["T"], "seed": it["seed"], "mode": "seq", "precision": "binary64",
           "pairs": f"random walks {WALK}" if walks else "arc draws",
           "auc_uc": oracle.auc(m.scores(hs, hd, 2), m.scores(hs, neg, 2)),
           "auc_uu": oracle.auc(oracle.pair_scores(m.U, m.U, hs, hd), oracle.pair_scores(m.U, m.U, hs, neg)),
           "command": f"python tests/golden/make_golden.py {sys.argv[1]}"}
    res["oracle_seconds"] = round(time.time() - t0, 1)
    with open(os.path.join(HERE, out), "w") as f:
        json.dump(res, f, indent=1)
    print(json.dumps(res))


def _sbm_run(args):
    pairs, storage, train_seed = args
    from synth.labels import node_classification_f1, sbm_workload
    g, labels, c = sbm_workload()
    tb = oracle.Tables(g.n, g.src, g.dst, g.w)
    m = oracle.Model(tb, d=c["d"], K=c["K"], orders=c["orders"], T=c["T"], seed=train_seed, eta0=c["eta0"],
                     storage=storage)
    wg = oracle.WalkGraph(tb, **WALK) if pairs in ("walks", "pool") else None
    m.train(0, c["T"], "seq", walks=wg, pool=oracle.pool_size(c["T"]) if pairs == "pool" else 0)
    return pairs, storage, train_seed, node_classification_f1(m.U, labels, c["split_seed"])


def run_sbm_f1(out: str, kinds=("arcs", "walks")):
    """Node-classification Micro/Macro-F1 (Sec. V-A) of the labelled workload's vertex
    embeddings U, trained by the oracle (SEQ) with arc-draw pairs and with random-walk
    pairs, with binary64 tables and with bfloat16 table storage (the precision
    extension's reference); the workload's training seed, plus two more seeds whose
    spread sizes the tolerance of the GPU comparison."""
    from concurrent.futures import ProcessPoolExecutor
    from synth.labels import SBM, sbm_workload
    t0 = time.time()
    g, _, c = sbm_workload()
    seeds = [c["train_seed"], 70, 71]
    jobs = [(p, st, s) for st in ("binary64", "bf16") for p in kinds for s in seeds]
    with ProcessPoolExecutor(max_workers=min(len(jobs), os.cpu_count() or 1)) as ex:
        results = list(ex.map(_sbm_run, jobs))
    res = {"workload": "synth.labels.SBM", "config": SBM, "n": g.n, "m": g.m, "T": c["T"], "mode": "seq",
           "precision": "binary64 arithmetic; binary64 tables (arcs, walks, pool) or bfloat16 tables (arcs_bf16, "
                        "walks_bf16: nearest-rounded initial values, stochastically rounded writes)",
           "walk": WALK, "command": f"python tests/golden/make_golden.py {sys.argv[1]}"}
    if "pool" in kinds:
        res["pool_pairs"] = oracle.pool_size(c["T"])
    for storage in ("binary64", "bf16"):
        for pairs in kinds:
            rows = {s: f for p, st, s, f in results if p == pairs and st == storage}
            mi = [rows[s][0] for s in seeds]
            ma = [rows[s][1] for s in seeds]
            key = pairs if storage == "binary64" else pairs + "_bf16"
            res[key] = {"micro": rows[c["train_seed"]][0], "macro": rows[c["train_seed"]][1],
                        "micro_by_seed": dict(zip(map(str, seeds), mi)),
                        "macro_by_seed": dict(zip(map(str, seeds), ma)),
                        "sd_micro": float(np.std(mi, ddof=1)), "sd_macro": float(np.std(ma, ddof=1))}
    res["oracle_seconds"] = round(time.time() - t0, 1)
    with open(os.path.join(HERE, out), "w") as f:
        json.dump(res, f, indent=1)
    print(json.dumps(res))


if __name__ == "__main__":
    which = sys.argv[1]
    if which == "c1_auc":
        run_auc("C1", orders=2, T=CONFIGS["C1"]["T"], d=CONFIGS["C1"]["d"], out="c1_oracle_auc.json")
    elif which == "c2_auc":
        run_auc("C2", orders=3, T=CONFIGS["C2"]["T"], d=CONFIGS["C2"]["d"], out="c2_oracle_auc.json")
    elif which == "batch6_auc":
        run_batch6("batch6_oracle_auc.json")
    elif which == "batch6_bf16_auc":
        run_batch6("batch6_oracle_bf16_auc.json", storage="bf16")
    elif which == "mid_auc":
        run_mid("mid_oracle_auc.json")
    elif which == "c2_walk_auc":
        run_auc("C2", orders=3, T=CONFIGS["C2"]["T"], d=CONFIGS["C2"]["d"], out="c2_walk_oracle_auc.json",
                walks=True)
    elif which == "mid_walk_auc":
        run_mid("mid_walk_oracle_auc.json", walks=True)
    elif which == "sbm_f1":
        run_sbm_f1("sbm_oracle_f1.json")
    elif which == "c2_pool_auc":
        run_auc("C2", orders=3, T=CONFIGS["C2"]["T"], d=CONFIGS["C2"]["d"], out="c2_pool_oracle_auc.json",
                pool=True)
    elif which == "sbm_pool_f1":
        run_sbm_f1("sbm_pool_oracle_f1.json", kinds=("pool",))
    else:
        raise SystemExit(__doc__)
