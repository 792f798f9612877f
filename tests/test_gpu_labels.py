"""Node-classification quality (Sec. V-A: one-vs-rest logistic regression on 10 % of the
labels, Micro- and Macro-F1) of embeddings trained on the GPU, against the oracle's, on
the labelled stand-in graph (a stochastic block model; the paper's labelled datasets are
not available).

The bar: the GPU's F1 (Hogwild, concurrent) within max(0.01, 3 sd) of the oracle's (SEQ)
with the same table storage, on the same pairs, the same training seed and the same
label split, sd being the spread of the oracle's own F1 over three training seeds
(stored with the reference: about 0.0015 with arc draws, 0.006 with walk pairs, whose
pairs change with the seed as whole walks).  Pairs from a pair pool (Sec. IV-C,
Augmented-Pair) are held to the oracle's pool runs the same way.  bfloat16 tables are held to the oracle run
with bfloat16 storage (every write stochastically rounded), the precision extension's
reference; the stored binary64 value is printed beside it.
"""
import json
import os

import pytest

from synth.labels import node_classification_f1, sbm_workload

from gpu_util import trainer_for

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")

def _bar(ref, key):
    return max(0.01, 3.0 * ref["sd_" + key])



@pytest.mark.parametrize("pairs", ["arcs", "walks", "pool"])
@pytest.mark.parametrize("dtype", ["fp32", "bf16"])
def test_node_classification_f1_matches_oracle(dtype, pairs):
    import paper_2604_09419_amd as lh
    gold = json.load(open(os.path.join(GOLDEN, "sbm_oracle_f1.json")))
    if pairs == "pool":
        gold.update(json.load(open(os.path.join(GOLDEN, "sbm_pool_oracle_f1.json"))))
    g, labels, c = sbm_workload()
    assert (g.n, g.m, c["T"]) == (gold["n"], gold["m"], gold["T"])
    tr = trainer_for(g, d=c["d"], K=c["K"], orders=c["orders"], dtype=dtype, seed=c["train_seed"],
                     total_samples=c["T"], eta0=c["eta0"])
    if pairs in ("walks", "pool"):
        w = gold["walk"]
        tr.build_walks(walk_length=w["L"], window=w["W"], walks_per_batch=w["Bw"])
    if pairs == "pool":
        assert tr.build_pool() == gold["pool_pairs"]
    tr.train_steps(0, c["T"])
    tr.check()
    micro, macro = node_classification_f1(tr.read(lh.LH_TABLE_U).cpu().numpy(), labels, c["split_seed"])
    ref = gold[pairs if dtype == "fp32" else pairs + "_bf16"]
    print(f"SBM {dtype} {pairs}: micro-F1 {micro:.4f} (oracle {ref['micro']:.4f}, seed sd {ref['sd_micro']:.4f}; "
          f"binary64 oracle {gold[pairs]['micro']:.4f}) macro-F1 {macro:.4f} (oracle {ref['macro']:.4f})", flush=True)
    assert abs(micro - ref["micro"]) <= _bar(ref, "micro") and abs(macro - ref["macro"]) <= _bar(ref, "macro")
    tr.close()
