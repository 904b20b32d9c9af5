"""GPU parity of the CKKS horizontal path against the oracle (oracle/ckks.py):
encryption, addition and decryption residues bit-exact given the same seeded
keys and randomness; encoding and decoding within the stated tolerances; a
horizontal round (5 clients, G and H vectors of 7,680 values) within the
worst-case noise bound."""
import functools
import sys

import numpy as np
import pytest

import oracle.ckks as C

pytestmark = pytest.mark.gpu
KEY_SEED = 11


def say(msg):
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ck():
    import torch
    assert torch.cuda.is_available()
    from paper_2504_03909_amd import ckks
    return ckks


@functools.lru_cache(maxsize=None)
def oracle_keys(log_n):
    return C.keygen(C.Params(log_n, 40), KEY_SEED)


def host(t):
    import torch
    torch.cuda.synchronize()
    return t.cpu().numpy().view(np.uint32)


def rns_tensor(polys, primes):
    import torch
    arr = np.array([[[int(c) % q for c in p] for q in primes] for p in polys], dtype=np.uint64).astype(np.uint32)
    return torch.from_numpy(arr.view(np.int32)).cuda()


@pytest.mark.parametrize("log_n", [12, 13, 14])
def test_encrypt_add_decrypt_bit_exact(ck, log_n):
    say(f"ckks encrypt/add/decrypt log_n={log_n}")
    ctx = ck.Context(log_n, 40, KEY_SEED)
    keys = oracle_keys(log_n)
    primes = keys.params.primes
    assert ctx.primes == primes and ctx.n == 1 << log_n
    rng = np.random.default_rng(log_n)
    n = 1 << log_n
    msgs = [[int(x) for x in rng.integers(-(1 << 50), 1 << 50, size=n)] for _ in range(2)]
    pt = rns_tensor(msgs, primes)
    ct = ctx.encrypt(pt, seed=7, offset=5)
    got = host(ct)
    for t in range(2):
        c0, c1 = C.encrypt(keys, C.to_rns(msgs[t], primes), seed=7, index=5 + t)
        assert np.array_equal(got[t, 0], np.array(c0, dtype=np.uint32)), t
        assert np.array_equal(got[t, 1], np.array(c1, dtype=np.uint32)), t
    dec = host(ctx.decrypt(ct))
    for t in range(2):
        want = C.decrypt(keys, (got[t, 0].tolist(), got[t, 1].tolist()))
        assert np.array_equal(dec[t], np.array(want, dtype=np.uint32))
    s = ctx.add(ct[0:1], ct[1:2])
    wa = C.add((got[0, 0].tolist(), got[0, 1].tolist()), (got[1, 0].tolist(), got[1, 1].tolist()), primes)
    assert np.array_equal(host(s)[0, 0], np.array(wa[0], dtype=np.uint32))
    assert np.array_equal(host(s)[0, 1], np.array(wa[1], dtype=np.uint32))
    if log_n <= 12:  # the exact-noise identity (schoolbook products: small N only)
        back = C.from_rns(dec[0].tolist(), primes)
        assert [b - m for b, m in zip(back, msgs[0])] == C.fresh_noise(keys.params, KEY_SEED, 7, 5)


@pytest.mark.parametrize("log_n,n_values", [(12, 2048), (12, 1000), (14, 7680)])
def test_encode_decode_match_oracle(ck, log_n, n_values):
    import torch
    say(f"ckks encode/decode log_n={log_n} n={n_values}")
    ctx = ck.Context(log_n, 40, KEY_SEED)
    p = C.Params(log_n, 40)
    rng = np.random.default_rng(n_values)
    z = rng.normal(0, 100, size=n_values)
    pt = ctx.encode(torch.from_numpy(z[None]).cuda())
    got = C.from_rns(host(pt)[0].tolist(), p.primes)
    want = C.encode(z, p)
    # both sides round double-precision sums of ~2^47-sized terms: a few units
    assert max(abs(g - w) for g, w in zip(got, want)) <= 8
    back = host(ctx.decode(pt, n_values)).view(np.float64)[0]
    assert np.max(np.abs(back - z)) <= 1e-6
    ob = C.decode(want, p, min(n_values, 512))
    assert np.max(np.abs(back[:512] - ob)) <= 1e-6


def test_horizontal_round(ck):
    """5 clients, local G and H histograms of 7,680 values (e.g. 30 features x
    256 bins), log_n = 14: encrypt, server sum, decrypt, decode."""
    import torch
    say("ckks horizontal round")
    ctx = ck.Context(14, 40, KEY_SEED)
    rng = np.random.default_rng(1)
    clients, length = 5, 7680
    G = rng.normal(0, 200, size=(clients, length))
    H = rng.uniform(0, 500, size=(clients, length))
    z = torch.from_numpy(np.concatenate([G, H])).cuda()          # [2 clients, ...]
    ct = ctx.encrypt(ctx.encode(z), seed=99)                      # client c: rows c (G) and clients + c (H)
    acc = ct[[0, clients]].clone()
    for c in range(1, clients):
        acc = ctx.add(acc, ct[[c, clients + c]].contiguous())
    out = host(ctx.decode(ctx.decrypt(acc), length)).view(np.float64)
    err = np.abs(out - np.stack([G.sum(0), H.sum(0)]))
    # worst case per client: encoding rounding N/2 plus N * 21 (2N + 1) of
    # noise, over the scale
    n = ctx.n
    bound = clients * (n / 2 + n * 21 * (2 * n + 1)) / 2 ** 40
    assert err.max() <= bound, (err.max(), bound)
    assert err.max() <= 1e-4   # the typical size, far inside the bound
