"""GPU tests of batched aggregation: captured plans (HIP graphs), the
autotuner, many uneven jobs in one launch, and a depth-6 tree at full size.
Expected values come from the oracle (bit-exact ciphertexts through the
closed form prod E(m_i; r_i) = E(sum m_i; prod r_i)) and from exact integer
sums of the oracle's encoding (decrypted histograms)."""
import functools
import sys

import numpy as np
import pytest

import oracle.paillier as P
from synth import workloads as W

pytestmark = pytest.mark.gpu


def say(msg):
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def he():
    import torch
    assert torch.cuda.is_available()
    from paper_2504_03909_amd import he as H
    return H


@functools.lru_cache(maxsize=None)
def keys(bits, seed):
    from paper_2504_03909_amd import he as H
    p, q = P.keygen(bits, seed)
    return P.PrivateKey(p, q), H.Key.from_primes(bits, p, q)


def dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def host(t):
    import torch
    torch.cuda.synchronize()
    return t.cpu().numpy()


def encode_all(g):
    return np.array([P.encode(float(x)) for x in g.reshape(-1)], dtype=np.int64).reshape(g.shape)


def plain_sums(m, idx, bins_f, K):
    """Exact sums per bin (|sum| < 2^53, so float64 accumulation is exact)."""
    return np.stack([np.rint(np.bincount(bins_f[idx], weights=m[idx, t].astype(np.float64),
                                         minlength=K)).astype(np.int64) for t in range(2)], axis=-1)


def closed_form(pk, bits, r_seed, m, members, t):
    rp = 1
    for i in members:
        rp = rp * P.seeded_r(pk.n, bits, r_seed, 2 * int(i) + t) % pk.n
    return P.encrypt(pk, int(m[members, t].sum()), rp) if len(members) else 1


# ------------------------------------------------------------ small cases
@pytest.fixture(scope="module")
def small(he):
    bits, M, r_seed = 1024, 3000, 91
    sk, k = keys(bits, 1)
    s = W.streams(7)
    g = W.gradients(M, s[1])
    m = encode_all(g)
    ct = he.encrypt(k, dev(m.reshape(-1)), seed=r_seed).view(M, 2, -1)
    tables = W.bins_tables(M, 24, (16, 64, 256), s[2])
    shapes = W.batched_jobs(9, s[5], M, min_samples=1, max_samples=M, min_features=1, max_features=24)
    return dict(bits=bits, M=M, r_seed=r_seed, sk=sk, k=k, m=m, ct=ct, tables=tables, shapes=shapes)


def make_jobs(he, small_or_tables, shapes):
    tables = small_or_tables
    dt = {b: dev(t) for b, t in tables.items()}
    jobs = []
    for sh in shapes:
        B, F, f0 = sh["n_bins"], sh["n_features"], sh["f0"]
        jobs.append(he.Job(dev(sh["sample_idx"].view(np.int32)), dt[B][f0:f0 + F], B))
    return jobs


def check_job(he, c, sh, hist, n_slots=3):
    """Decrypted sums for every slot, closed-form ciphertexts for a few."""
    B, F, f0 = sh["n_bins"], sh["n_features"], sh["f0"]
    tab = c["tables"][B][f0:f0 + F]
    idx = sh["sample_idx"].astype(np.int64)
    dm, _, ovf = he.decrypt(c["k"], hist)
    dm = host(dm)
    for f in range(F):
        assert np.array_equal(dm[f], plain_sums(c["m"], idx, tab[f], B)), f
    h = host(hist)
    rng = np.random.default_rng(len(idx))
    pk = c["sk"].public
    for _ in range(n_slots):
        f, b, t = int(rng.integers(F)), int(rng.integers(B)), int(rng.integers(2))
        members = idx[tab[f][idx] == b]
        assert he.limbs_to_ints(h[f, b, t][None])[0] == closed_form(pk, c["bits"], c["r_seed"], c["m"], members, t)


def test_batched_equals_per_job_and_oracle(he, small):
    import torch
    say("batched vs per-job (small)")
    c = small
    jobs = make_jobs(he, c["tables"], c["shapes"])
    he.hist_aggregate(c["k"], c["ct"], jobs)
    batched = [j.hist.clone() for j in jobs]
    for j, sh, hb in zip(jobs, c["shapes"], batched):
        (alone,) = he.hist_aggregate(c["k"], c["ct"], [he.Job(j.sample_idx, j.bins, j.n_bins)])
        assert torch.equal(alone, hb)
        check_job(he, c, sh, hb)


def test_plan_replays_match_direct(he, small):
    """A captured plan, replayed several times with other device work and
    host synchronisation between replays, rewrites the same histograms."""
    import torch
    say("plan replay (small)")
    c = small
    jobs = make_jobs(he, c["tables"], c["shapes"])
    he.hist_aggregate(c["k"], c["ct"], jobs)
    want = [j.hist.clone() for j in jobs]
    jobs2 = make_jobs(he, c["tables"], c["shapes"])
    plan = he.HistPlan(c["k"], c["ct"], jobs2, chunk=7, split=1)
    for rep in range(3):
        for h in plan.hists:
            h.fill_(-1)
        he.encrypt(c["k"], torch.arange(64, dtype=torch.int64, device="cuda"), seed=rep)  # eager work
        torch.cuda.synchronize()
        plan.launch()
        torch.cuda.synchronize()
        for h, w in zip(plan.hists, want):
            assert torch.equal(h, w), rep
    # Montgomery-form input in a plan
    ctm = he.to_mont(c["k"], c["ct"])
    jobs3 = make_jobs(he, c["tables"], c["shapes"])
    plan2 = he.HistPlan(c["k"], ctm, jobs3, form=he.HE_FORM_MONT)
    plan2.launch()
    for h, w in zip(plan2.hists, want):
        assert torch.equal(h, w)


def test_autotune_keeps_results(he, small):
    import torch
    say("autotune (small)")
    c = small
    jobs = make_jobs(he, c["tables"], c["shapes"])
    he.hist_aggregate(c["k"], c["ct"], jobs, chunk=64)
    want = [j.hist.clone() for j in jobs]
    chunk, split, lanes, waves, ms = he.hist_autotune(c["k"], c["ct"], jobs)
    assert chunk in (16, 32, 64, 128, 256, 512) and split in (1, 2) and ms > 0
    assert lanes in (8, 16) and waves in (0, 2, 3, 4)
    for h, w in zip([j.hist for j in jobs], want):
        assert torch.equal(h, w)
    he.hist_aggregate(c["k"], c["ct"], jobs)  # chunk 0 -> tuned shape
    for h, w in zip([j.hist for j in jobs], want):
        assert torch.equal(h, w)


@pytest.mark.parametrize("split", [1, 2])
@pytest.mark.parametrize("chunk", [1, 5, 300])
def test_split_and_chunk_variants(he, small, split, chunk):
    import torch
    say(f"split={split} chunk={chunk}")
    c = small
    jobs = make_jobs(he, c["tables"], c["shapes"][:4])
    he.hist_aggregate(c["k"], c["ct"], jobs, chunk=64)
    want = [j.hist.clone() for j in jobs]
    plan = he.HistPlan(c["k"], c["ct"], make_jobs(he, c["tables"], c["shapes"][:4]), chunk=chunk, split=split)
    plan.launch()
    for h, w in zip(plan.hists, want):
        assert torch.equal(h, w)


# ------------------------------------------------------- full-size shapes
@pytest.mark.parametrize("bits,seed", [(1024, 1), (2048, 2)])
def test_final_join_of_runs(he, bits, seed):
    """Bins holding exactly 0 to 100 samples, aggregated with one partial per
    sample (chunk 1) and per three, so that the final kernel joins every
    number of runs (1, 2, 4, 8) with run lengths on both sides of the powers
    of two; three features hold the same counts in different bins (other
    ranks), and a second job in the same launch has 5 bins (ranks past its
    bins are skipped).  Every decrypted sum is exact, sampled ciphertexts
    equal the closed form, the counters equal the algorithm's count, and the
    histograms equal those of the default chunk."""
    import torch
    say(f"final join of runs, {bits}-bit")
    counts = [0, 1, 2, 3, 4, 5, 6, 7, 8, 9, 11, 15, 16, 17, 31, 32, 33, 35, 63, 64, 65, 100]
    B, F, r_seed = len(counts), 3, 17
    M = sum(counts)
    sk, k = keys(bits, seed)
    rng = np.random.default_rng(bits + 3)
    base = np.repeat(np.arange(B), counts)
    tab = np.stack([rng.permutation(B)[base][rng.permutation(M)] for _ in range(F)]).astype(np.uint8)
    m = encode_all(W.gradients(M, W.streams(8)[1]))
    ct = he.encrypt(k, dev(m.reshape(-1)), seed=r_seed).view(M, 2, -1)
    idx2 = np.sort(rng.choice(M, size=300, replace=False)).astype(np.int64)
    tab2 = (tab % 5).astype(np.uint8)
    c = dict(bits=bits, sk=sk, k=k, m=m, r_seed=r_seed)

    def jobs():
        return [he.Job(dev(np.arange(M, dtype=np.int32)), dev(tab), B),
                he.Job(dev(idx2.astype(np.int32)), dev(tab2), 5)]

    hs64, _ = he.hist_aggregate_counted(k, ct, jobs(), chunk=64)
    for chunk in (1, 3):
        hs, cnt = he.hist_aggregate_counted(k, ct, jobs(), chunk=chunk, split=2)
        for h, h64 in zip(hs, hs64):
            assert torch.equal(h, h64), chunk
        real = conv = 0
        for (ix, tb, nb) in ((np.arange(M), tab, B), (idx2, tab2, 5)):
            for f in range(F):
                real += 2 * (ix.size - np.unique(tb[f][ix]).size)
            conv += F * nb * 2
        got = host(cnt).tolist()
        assert got[0] == real and got[2] == conv and got[1] >= real + conv, (chunk, got, real, conv)
    pk = sk.public
    for (ix, tb, nb, h) in ((np.arange(M), tab, B, hs[0]), (idx2, tab2, 5, hs[1])):
        dm, _, ovf = he.decrypt(k, h)
        dm = host(dm)
        assert int(host(ovf)[0]) == 0
        for f in range(F):
            assert np.array_equal(dm[f], plain_sums(m, ix, tb[f], nb)), (nb, f)
    hh = host(hs[0])
    for f, cnt_want, t in ((0, 100, 0), (1, 65, 1), (2, 17, 0), (0, 8, 1), (1, 1, 0), (2, 0, 1)):
        b = int(np.flatnonzero(np.bincount(tab[f], minlength=B) == cnt_want)[0])
        members = np.flatnonzero(tab[f] == b)
        assert he.limbs_to_ints(hh[f, b, t][None])[0] == closed_form(pk, bits, r_seed, m, members, t), (f, b, t)


def test_batched_64_jobs_2048(he):
    """64 uneven jobs (|S| log-uniform in [1e3, 2e5], F in [8, 128],
    B in {16, 64, 256}) over a pool of 200,000 samples, 2048-bit key: one
    batched launch equals one launch per job and the oracle's sums."""
    import torch
    say("64 jobs over 200k pool, 2048-bit")
    bits, M, r_seed = 2048, 200_000, 404
    sk, k = keys(bits, 2)
    s = W.streams(4)
    g = W.gradients(M, s[1])
    m = encode_all(g)
    ct = he.encrypt(k, dev(m.reshape(-1)), seed=r_seed).view(M, 2, -1)
    ctm = he.to_mont(k, ct)
    tables = W.bins_tables(M, 128, (16, 64, 256), s[2])
    shapes = W.batched_jobs(64, s[5], M)
    jobs = make_jobs(he, tables, shapes)
    he.hist_aggregate(k, ctm, jobs, form=he.HE_FORM_MONT)
    batched = [j.hist.clone() for j in jobs]
    for j, hb in zip(jobs, batched):
        (alone,) = he.hist_aggregate(k, ctm, [he.Job(j.sample_idx, j.bins, j.n_bins)], form=he.HE_FORM_MONT)
        assert torch.equal(alone, hb)
    # every work shape the autotuner can pick gives the same histograms
    for lanes in (16, 8):
        for split, chunk in ((2, 128), (1, 64)):
            for waves in (0, 4, 3, 2):
                say(f"64 jobs at lanes={lanes} split={split} chunk={chunk} waves={waves}")
                hs, cnt = he.hist_aggregate_counted(k, ctm, make_jobs(he, tables, shapes), form=he.HE_FORM_MONT,
                                                    chunk=chunk, split=split, lanes=lanes, waves=waves)
                assert all(torch.equal(h, hb) for h, hb in zip(hs, batched)), (lanes, split, chunk, waves)
    c = dict(bits=bits, M=M, r_seed=r_seed, sk=sk, k=k, m=m, ct=ct, tables=tables)
    order = np.argsort([sh["sample_idx"].size for sh in shapes])
    for n, ji in enumerate(order):
        # every job's decrypted sums; closed-form ciphertexts on the smaller half
        check_job(he, c, shapes[ji], batched[ji], n_slots=2 if n < 32 else 0)


def test_tree_depth6_full_size(he):
    """2048-bit key, 1,000,000 samples, 64 features x 256 Zipf bins, depth-6
    tree (63 nodes, seeded splits): one job per launch, one captured plan per
    level and the sibling mode (smaller child aggregated, larger one the
    parent divided by it) give identical histograms; every node's decrypted histogram
    equals the oracle's sums; sampled slots are bit-exact in closed form."""
    import torch
    from paper_2504_03909_amd import pipeline
    say("depth-6 tree, 1M samples, 64 x 256, 2048-bit")
    bits, M, J, K, r_seed = 2048, 1_000_000, 64, 256, 606
    sk, k = keys(bits, 2)
    s = W.streams(3)
    g = W.gradients(M, s[1])
    bins = W.bins_zipf(J, M, K, s[2])
    levels = W.tree_levels(M, 6, s[4])
    assert sum(len(l) for l in levels) == 63
    res = pipeline.encrypt_gradients(k, dev(g), r_seed)
    bins_d = dev(bins)
    lv_d = [[dev(n.view(np.int32)) for n in lvl] for lvl in levels]
    plain = pipeline.aggregate_levels(res, lv_d, bins_d, K, mode="per_node")
    graph = pipeline.aggregate_levels(res, lv_d, bins_d, K, mode="per_level_graph")
    sib = pipeline.aggregate_levels(res, lv_d, bins_d, K, mode="sibling")
    for other in (graph, sib):
        for la, lb in zip(plain.hists, other.hists):
            for a, b in zip(la, lb):
                assert torch.equal(a, b)
    del graph, sib
    dec = pipeline.decrypt_levels(k, plain)
    m = np.rint(g * 2.0 ** 32).astype(np.int64)
    rng = np.random.default_rng(0)
    pick = rng.choice(M, size=2000, replace=False)
    assert all(m[i, t] == P.encode(float(g[i, t])) for i in pick for t in range(2))
    for lvl, dl in zip(levels, dec):
        for node, dm in zip(lvl, dl):
            dmh = host(dm)
            idx = node.astype(np.int64)
            for f in range(J):
                assert np.array_equal(dmh[f], plain_sums(m, idx, bins[f], K))
    # closed-form ciphertexts on a depth-5 node (~30k samples)
    pk = sk.public
    node = levels[5][3].astype(np.int64)
    hh = host(plain.hists[5][3])
    for f, t in ((0, 0), (17, 1), (63, 0)):
        b = int(np.bincount(bins[f][node], minlength=K).argmax())
        members = node[bins[f][node] == b]
        assert he.limbs_to_ints(hh[f, b, t][None])[0] == closed_form(pk, bits, r_seed, m, members, t)


@pytest.mark.parametrize("split", [1, 2])
@pytest.mark.parametrize("chunk", [1, 7, 64, 5000])
def test_work_counters(he, small, split, chunk):
    """The device's count of Montgomery products that join two real partial
    products equals, for every (job, feature, slot), |S| minus the number of
    non-empty bins; one conversion per histogram entry; executed products
    (padding included) bound it from above; the histograms are unchanged."""
    import torch
    say(f"work counters chunk={chunk} split={split}")
    c = small
    jobs = make_jobs(he, c["tables"], c["shapes"])
    he.hist_aggregate(c["k"], c["ct"], jobs, chunk=64)
    want = [j.hist.clone() for j in jobs]
    jobs2 = make_jobs(he, c["tables"], c["shapes"])
    hists, cnt = he.hist_aggregate_counted(c["k"], c["ct"], jobs2, chunk=chunk, split=split)
    for h, w in zip(hists, want):
        assert torch.equal(h, w)
    real = conv = 0
    for sh in c["shapes"]:
        B, F, f0 = sh["n_bins"], sh["n_features"], sh["f0"]
        idx = sh["sample_idx"].astype(np.int64)
        for f in range(F):
            nonempty = np.unique(c["tables"][B][f0 + f][idx]).size if idx.size else 0
            real += 2 * (idx.size - nonempty)
        conv += F * B * 2
    got = host(cnt).tolist()
    assert got[0] == real and got[2] == conv
    assert got[1] >= real + conv
