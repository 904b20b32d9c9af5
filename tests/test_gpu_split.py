"""GPU parity of split finding from decrypted histograms against the oracle
(oracle/split.py): per-node and per-feature best splits, gains equal as
IEEE doubles, bins/features/left sums exact; the sibling form hist - minus;
ties, inadmissible features and single-bin features."""
import sys

import numpy as np
import pytest

from oracle import split as S

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


def host(t):
    import torch
    torch.cuda.synchronize()
    return t.cpu().numpy()


def random_hist(rng, nodes, F, B, scale=40):
    g = rng.integers(-(1 << scale), 1 << scale, size=(nodes, F, B))
    h = rng.integers(0, 1 << scale, size=(nodes, F, B))
    h[rng.random((nodes, F, B)) < 0.2] = 0          # empty bins
    return np.stack([g, h], axis=-1).astype(np.int64)


def check(res, hist, frac, lam, gamma, mcw):
    per_feat, per_node = S.best_splits(hist.tolist(), frac, lam, gamma, mcw)
    gain, feat, b = host(res["gain"]), host(res["feature"]), host(res["bin"])
    gl, hl = host(res["g_left"]), host(res["h_left"])
    for i, want in enumerate(per_node):
        assert (gain[i] == want.gain) or (np.isinf(gain[i]) and np.isinf(want.gain)), (i, gain[i], want.gain)
        assert (feat[i], b[i]) == (want.feature, want.bin), i
        if want.bin >= 0:
            assert (gl[i], hl[i]) == (want.g_left, want.h_left)
    pf = res["per_feature"]
    fg, fb = host(pf["gain"]), host(pf["bin"])
    for i, row in enumerate(per_feat):
        for f, want in enumerate(row):
            assert fb[i, f] == want.bin and (fg[i, f] == want.gain or (np.isinf(fg[i, f]) and np.isinf(want.gain)))


@pytest.mark.parametrize("B", [1, 2, 17, 64, 256])
@pytest.mark.parametrize("lam,gamma,mcw", [(1.0, 0.0, 1.0), (0.0, 0.25, 0.0), (3.5, 0.0, 50.0)])
def test_split_matches_oracle(he, B, lam, gamma, mcw):
    import torch
    say(f"split B={B} lam={lam} gamma={gamma} mcw={mcw}")
    rng = np.random.default_rng(B * 7 + int(lam * 10))
    hist = random_hist(rng, 6, 9, B)
    res = he.split_find(torch.from_numpy(hist).cuda(), lam=lam, gamma=gamma, min_child_weight=mcw,
                        per_feature=True)
    check(res, hist, 32, lam, gamma, mcw)


def test_split_sibling_form_and_derived(he):
    import torch
    say("split parent - child")
    rng = np.random.default_rng(5)
    child = random_hist(rng, 4, 5, 64, scale=36)
    parent = child + random_hist(rng, 4, 5, 64, scale=36)
    derived = torch.empty(parent.shape, dtype=torch.int64, device="cuda")
    res = he.split_find(torch.from_numpy(parent).cuda(), minus=torch.from_numpy(child).cuda(), derived=derived,
                        per_feature=True)
    assert np.array_equal(host(derived), parent - child)
    check(res, parent - child, 32, 1.0, 0.0, 1.0)


def test_split_ties_and_inadmissible(he):
    import torch
    say("split ties")
    one = 1 << 32
    B = 8
    hist = np.zeros((2, 4, B, 2), dtype=np.int64)
    # node 0: features 1 and 3 identical and symmetric (bins 2 and 4 give the
    # same gain); feature 0 all empty (nothing admissible with lambda = 0)
    pat = np.array([[1, 1], [1, 1], [-3, 1], [0, 1], [0, 1], [3, 1], [-1, 1], [-1, 1]], dtype=np.int64) * one
    hist[0, 1] = pat
    hist[0, 3] = pat
    hist[0, 2] = pat // 2
    # node 1: everything empty
    res = he.split_find(torch.from_numpy(hist).cuda(), lam=0.0, min_child_weight=0.0, per_feature=True)
    check(res, hist, 32, 0.0, 0.0, 0.0)
    assert host(res["feature"])[0] == 1 and host(res["feature"])[1] == -1
    assert np.isinf(host(res["gain"])[1]) and host(res["gain"])[1] < 0


def test_split_end_to_end_after_decrypt(he):
    """1024-bit key: encrypt, aggregate a node, decrypt, split on the GPU ==
    the oracle's split of the oracle's exact plaintext histogram."""
    import torch
    import oracle.paillier as P
    from synth import workloads as W
    say("split end to end")
    p, q = P.keygen(1024, 1)
    k = he.Key.from_primes(1024, p, q)
    s = W.streams(12)
    M, J, K = 3000, 6, 32
    g = W.gradients(M, s[1])
    bins = W.bins_zipf(J, M, K, s[2])
    m = he.encode(torch.from_numpy(g.reshape(-1)).cuda())
    ct = he.encrypt(k, m, seed=5).view(M, 2, -1)
    idx = torch.arange(0, M, 2, dtype=torch.int32, device="cuda")
    (hist,) = he.hist_aggregate(k, ct, [he.Job(idx, torch.from_numpy(bins).cuda(), K)])
    dm, _, _ = he.decrypt(k, hist)
    res = he.split_find(dm.view(1, J, K, 2), per_feature=True)
    mo = np.array([[P.encode(float(x)) for x in row] for row in g], dtype=np.int64)
    plain = P.plaintext_histogram(mo.tolist(), range(0, M, 2), bins.tolist(), J, K)
    check(res, np.array([plain], dtype=np.int64), 32, 1.0, 0.0, 1.0)


def test_tree_round_sibling_modes_agree(he):
    """1024-bit key, 4,000 samples, 6 features x 32 Zipf bins, depth-4 tree:
    direct, encrypted-sibling and plaintext-sibling rounds (the last also with
    packed decryption) give identical plaintext histograms and splits; every node's split equals the oracle's
    split of its exact plaintext histogram."""
    import torch
    import oracle.paillier as P
    from paper_2504_03909_amd import pipeline
    from synth import workloads as W
    say("tree round, three sibling modes")
    p, q = P.keygen(1024, 1)
    k = he.Key.from_primes(1024, p, q)
    s = W.streams(13)
    M, J, K = 4000, 6, 32
    g = W.gradients(M, s[1])
    bins = W.bins_zipf(J, M, K, s[2])
    levels = W.tree_levels(M, 4, s[4])
    res = pipeline.encrypt_gradients(k, torch.from_numpy(g).cuda(), 99)
    bd = torch.from_numpy(bins).cuda()
    lv = [[torch.from_numpy(n.view(np.int32)).cuda() for n in lvl] for lvl in levels]
    runs = {mode: pipeline.tree_round(res, k, lv, bd, K, sibling=mode) for mode in (None, "encrypted", "plain")}
    runs["plain_packed"] = pipeline.tree_round(res, k, lv, bd, K, sibling="plain", packed=True)
    base = runs[None]
    for mode in ("encrypted", "plain", "plain_packed"):
        for a, b in zip(base.plain, runs[mode].plain):
            assert torch.equal(a, b), mode
        for sa, sb in zip(base.splits, runs[mode].splits):
            for key in ("gain", "feature", "bin", "g_left", "h_left"):
                assert torch.equal(sa[key], sb[key]), (mode, key)
    mo = np.array([[P.encode(float(x)) for x in row] for row in g], dtype=np.int64)
    for lvl, plain, sp in zip(levels, base.plain, base.splits):
        ph = host(plain)
        for i, node in enumerate(lvl):
            want = np.array(P.plaintext_histogram(mo.tolist(), node.tolist(), bins.tolist(), J, K), dtype=np.int64)
            assert np.array_equal(ph[i], want)
            _, per_node = S.best_splits([want.tolist()], 32, 1.0, 0.0, 1.0)
            assert host(sp["gain"])[i] == per_node[0].gain or (per_node[0].bin < 0)
            assert (host(sp["feature"])[i], host(sp["bin"])[i]) == (per_node[0].feature, per_node[0].bin)
