"""Full-size parity in the launch configuration the benchmark times
(graph-captured plan, autotuned config).

* 64M words: the whole permutation against the oracle's definition applied
  to every length list (the lists on host threads, a few seconds), besides
  the invariants that hold at any size (permutation, strict key order,
  bucket sizes equal the length histogram) and sampled positions against
  the oracle's definitional rank of a word (perm[rank(i)] == i).
* 4096 documents (about 31M words): every document against the oracle.
* The sorted text written in the sort's own pass (sw_plan_run_text): for the
  documents, byte for byte against the oracle's text; for 64M words, byte for
  byte against the oracle's writer applied to the order the invariants prove,
  equal to the permutation-based writer's output, and at sampled words equal
  to the word the oracle ranks there.
"""
import numpy as np
import pytest

from checks import check_invariants
from paper_1411_5283_amd import wordgen

pytestmark = pytest.mark.gpu


def _plan_sort(sw, wl, workload, text=False):
    """Sort through a plan (twice: a replay must give the same result); with
    text, also run the sort with the sorted text (line feeds) and return the
    text and the permutation-based writer's text of the same permutation."""
    import torch
    from paper_1411_5283_amd import tune
    saved = sw.get_config()
    tune.apply(workload)
    try:
        chars, offs, docs = sw.device_words(wl)
        perm = torch.empty(max(wl.n, 1), dtype=torch.int32, device="cuda")
        boff = torch.empty(wl.n_docs * 34, dtype=torch.int32, device="cuda")
        plan = sw.Plan(wl.n, wl.n_docs)
        texts = None
        try:
            for _ in range(2):
                plan.run(chars, offs, docs, wl.n_docs, wl.n, perm, boff)
                plan.status()
            if text:
                size = sw.text_size(wl, 10)
                out = torch.empty(size, dtype=torch.uint8, device="cuda")
                perm2 = torch.empty_like(perm)
                plan.run_text(chars, offs, docs, wl.n_docs, wl.n, perm2, boff, 10, out)
                plan.status()
                assert torch.equal(perm2, perm), "the text run sorted differently"
                ref = torch.empty(size, dtype=torch.uint8, device="cuda")
                st = torch.zeros(1, dtype=torch.int32, device="cuda")
                sw.materialize(chars, offs, docs, wl.n_docs if docs is not None else 1, wl.n, perm, boff, 10, ref, st)
                torch.cuda.synchronize()
                assert int(st.cpu()[0]) == 0
                texts = (out.cpu().numpy(), ref.cpu().numpy())
        finally:
            plan.close()
        res = (sw.to_u32(perm)[:wl.n], sw.to_u32(boff).reshape(wl.n_docs, 34))
        return res + (texts,) if text else res
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
def test_config4_full_against_oracle(gpu, oracle_mod):
    print("case config4 full 64M words", flush=True)
    wl = wordgen.config(4)
    perm, boff, (text, ref) = _plan_sort(gpu, wl, "c4", text=True)
    boff = boff[0]
    counts = oracle_mod.oracle_length_counts(wl.offsets)
    assert np.array_equal(np.diff(boff.astype(np.int64)), counts.astype(np.int64))
    check_invariants(wl.chars, wl.offsets, perm, boff)
    # the whole permutation against the oracle (its definition on every
    # length list, the lists on host threads): element by element
    eperm, eboff = oracle_mod.oracle_def_parallel(wl.chars, wl.offsets)
    assert np.array_equal(boff, eboff)
    bad = np.nonzero(perm != eperm)[0]
    assert bad.size == 0, "differs from the oracle at %d of %d positions" % (bad.size, wl.n)
    assert np.array_equal(text, ref), "text from the keys differs from the text from the permutation"
    # the invariants make perm the one sorted order; the oracle's writer lays
    # its words out on the host: the whole text, byte for byte
    etext = oracle_mod.oracle_materialize(wl.chars, wl.offsets, perm, 10)
    assert text.tobytes() == etext, "sorted text differs from the oracle's text of the verified order"
    # text position of sorted position k: the lengths before its bucket, then its rank in the bucket
    bo = boff.astype(np.int64)
    bucket_start = np.concatenate([[0], np.cumsum(np.diff(bo) * (np.arange(33) + 1))])
    rng = np.random.default_rng(4)
    for i in rng.integers(0, wl.n, 12):
        k = oracle_mod.oracle_rank(wl.chars, wl.offsets, int(i))
        assert perm[k] == i, (int(i), k)
        word = wl.chars[wl.offsets[i]:wl.offsets[i + 1]].tobytes()
        L = len(word)
        pos = int(bucket_start[L]) + (k - int(bo[L])) * (L + 1)
        assert text[pos:pos + L + 1].tobytes() == word + b"\n", (int(i), k)


@pytest.mark.timeout(1200)
def test_config3_full_every_document(gpu, oracle_mod):
    print("case config3 full 4096 documents", flush=True)
    wl = wordgen.config(3)
    perm, boff, (text, _) = _plan_sort(gpu, wl, "c3", text=True)
    eperm, eboff = oracle_mod.oracle_batch(wl.chars, wl.offsets, wl.doc_offsets, fn="oracle_def")
    assert np.array_equal(boff, eboff)
    bad = np.nonzero(perm != eperm)[0]
    assert bad.size == 0, "differs at %d positions" % bad.size
    etext = oracle_mod.oracle_materialize_batch(wl.chars, wl.offsets, wl.doc_offsets, eperm, 10)
    assert text.tobytes() == etext, "sorted text differs from the oracle's"
