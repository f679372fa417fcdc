"""Full-size parity in the launch configuration the benchmark times
(graph-captured plan, autotuned config).

* 64M words: the oracle cannot sort this, so the whole output is checked
  against invariants that hold at any size (permutation, strict key order,
  bucket sizes equal the length histogram) and sampled positions against
  the oracle's definitional rank of a word (perm[rank(i)] == i).
* 4096 documents (about 31M words): every document against the oracle.
"""
import numpy as np
import pytest

from checks import check_invariants
from paper_1411_5283_amd import wordgen

pytestmark = pytest.mark.gpu


def _plan_sort(sw, wl, workload):
    import torch
    from paper_1411_5283_amd import tune
    saved = sw.get_config()
    tune.apply(workload)
    try:
        chars, offs, docs = sw.device_words(wl)
        perm = torch.empty(max(wl.n, 1), dtype=torch.int32, device="cuda")
        boff = torch.empty(wl.n_docs * 34, dtype=torch.int32, device="cuda")
        plan = sw.Plan(wl.n, wl.n_docs)
        try:
            for _ in range(2):                       # a replay must give the same result
                plan.run(chars, offs, docs, wl.n_docs, wl.n, perm, boff)
                plan.status()
        finally:
            plan.close()
        return sw.to_u32(perm)[:wl.n], sw.to_u32(boff).reshape(wl.n_docs, 34)
    finally:
        sw.set_config(**saved)


@pytest.fixture(scope="module")
def gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1411_5283_amd as sw
    sw.lib()
    return sw


@pytest.mark.timeout(1200)
def test_config4_full_invariants_and_sampled_ranks(gpu, oracle_mod):
    print("case config4 full 64M words", flush=True)
    wl = wordgen.config(4)
    perm, boff = _plan_sort(gpu, wl, "c4")
    boff = boff[0]
    counts = oracle_mod.oracle_length_counts(wl.offsets)
    assert np.array_equal(np.diff(boff.astype(np.int64)), counts.astype(np.int64))
    check_invariants(wl.chars, wl.offsets, perm, boff)
    rng = np.random.default_rng(4)
    for i in rng.integers(0, wl.n, 12):
        k = oracle_mod.oracle_rank(wl.chars, wl.offsets, int(i))
        assert perm[k] == i, (int(i), k)


@pytest.mark.timeout(1200)
def test_config3_full_every_document(gpu, oracle_mod):
    print("case config3 full 4096 documents", flush=True)
    wl = wordgen.config(3)
    perm, boff = _plan_sort(gpu, wl, "c3")
    eperm, eboff = oracle_mod.oracle_batch(wl.chars, wl.offsets, wl.doc_offsets, fn="oracle_def")
    assert np.array_equal(boff, eboff)
    bad = np.nonzero(perm != eperm)[0]
    assert bad.size == 0, "differs at %d positions" % bad.size
