"""GPU parity of ciphertext packing against the oracle (oracle.paillier.pack
/ unpack): packed ciphertexts bit-exact for every slot count and ragged
tails, with a private or a public key; packed decryption equals plain
decryption; overflow of the top slot is flagged."""
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


def host(t):
    import torch
    torch.cuda.synchronize()
    return t.cpu().numpy()


def values(rng, count):
    v = rng.integers(-(1 << 62), 1 << 62, size=count, dtype=np.int64)
    v[:: max(1, count // 5)] = np.iinfo(np.int64).min
    v[1:: max(2, count // 3)] = np.iinfo(np.int64).max
    return v


@pytest.mark.parametrize("bits,seed", [(1024, 1), (2048, 2)])
@pytest.mark.parametrize("slots", [1, 2, 7, 0])
@pytest.mark.parametrize("count", [1, 40])
def test_pack_bit_exact_and_decrypts(he, bits, seed, slots, count):
    import torch
    sk, k = keys(bits, seed)
    pk = sk.public
    slots = slots or (bits - 1) // 64
    say(f"pack {bits} slots={slots} count={count}")
    rng = np.random.default_rng(bits + slots * 3 + count)
    v = values(rng, count)
    ct = he.encrypt(k, torch.from_numpy(v).cuda(), seed=77)
    packed, s = he.pack(k, ct, slots)
    assert s == slots and packed.shape[0] == -(-count // slots)
    cts = he.limbs_to_ints(host(ct))
    want = [P.pack(pk, cts[i:i + slots]) for i in range(0, count, slots)]
    assert he.limbs_to_ints(host(packed)) == want
    kpub = he.Key.public(bits, pk.n)
    packed_pub, _ = he.pack(kpub, ct, slots)
    assert torch.equal(packed_pub, packed)
    m, ovf = he.decrypt_packed(k, packed, count, slots)
    assert host(m).tolist() == v.tolist() and int(host(ovf)[0]) == 0


def test_pack_overflow_flagged(he):
    import torch
    say("pack overflow")
    sk, k = keys(1024, 1)
    pk = sk.public
    rng = np.random.default_rng(2)
    ms = [5, -7, (1 << 63) + 11, 3, 9, 1 << 70]   # top slots of the two packed ciphertexts out of range
    rs = W.random_units(pk.n, len(ms), rng)
    cts = [P.encrypt(pk, m, r) for m, r in zip(ms, rs)]
    ct = torch.from_numpy(he.ints_to_limbs(cts, 2 * k.limbs)).cuda()
    packed, _ = he.pack(k, ct, 3)
    m, ovf = he.decrypt_packed(k, packed, len(ms), 3)
    assert int(host(ovf)[0]) == 2
    assert host(m).tolist()[:2] == [5, -7] and host(m).tolist()[3:5] == [3, 9]


def test_pack_node_histogram_auto_slots(he):
    """A 2048-bit node histogram (32 features x 256 bins x g,h = 16,384
    ciphertexts) with the library's slot count: packed decryption equals
    plain decryption."""
    import torch
    say("pack node histogram, 2048-bit")
    sk, k = keys(2048, 2)
    s = W.streams(14)
    M, J, K = 20000, 32, 256
    g = W.gradients(M, s[1])
    bins = torch.from_numpy(W.bins_zipf(J, M, K, s[2])).cuda()
    m = he.encode(torch.from_numpy(g.reshape(-1)).cuda())
    ct = he.encrypt(k, m, seed=3).view(M, 2, -1)
    (hist,) = he.hist_aggregate(k, ct, [he.Job(torch.arange(M, dtype=torch.int32, device="cuda"), bins, K)])
    plain, _, _ = he.decrypt(k, hist)
    packed, slots = he.pack(k, hist)
    assert 1 <= slots <= 31
    mp, ovf = he.decrypt_packed(k, packed, hist.numel() // hist.shape[-1], slots)
    assert torch.equal(mp.view(plain.shape), plain) and int(host(ovf)[0]) == 0
