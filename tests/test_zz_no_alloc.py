"""The allocation-free decryption entry point (he_decrypt_noalloc) against
he_decrypt, through the C ABI: two calls in a row on the device's shared
scratch, the second smaller than the first, both bit-identical to
he_decrypt (signed plaintexts, raw plaintexts, overflow counts); the
plaintexts of the real encryptions are also checked against the values that
were encrypted.  Sizes beyond the scratch are refused before any device work.
"""
import sys

import numpy as np
import pytest

import oracle.paillier as P

pytestmark = pytest.mark.gpu


def say(msg):
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def setup():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    from paper_2504_03909_amd import he
    p, q = P.keygen(2048, 1)
    return he, he.Key.from_primes(2048, p, q), p * q


def _inputs(he, key, n, count, seed):
    """count ciphertexts: the first half encryptions of known int64 values
    (seeded r), the rest uniform residues mod n^2 (plaintexts mostly outside
    the int64 range, so the overflow count is exercised)."""
    import torch
    rng = np.random.default_rng(seed)
    n_enc = count // 2
    m = rng.integers(-(1 << 62), 1 << 62, size=n_enc, dtype=np.int64)
    m[:4] = [0, -1, (1 << 63) - 1, -(1 << 63)]
    ct_enc = he.encrypt(key, torch.from_numpy(m).cuda(), seed=seed)
    n2 = n * n
    vals = [int.from_bytes(rng.bytes(520), "little") % n2 for _ in range(count - n_enc)]
    ct_rand = torch.from_numpy(he.ints_to_limbs(vals, 2 * key.limbs).view(np.int32)).cuda()
    return torch.cat([ct_enc.view(n_enc, -1), ct_rand.view(count - n_enc, -1)]).contiguous(), m


def _check_call(he, key, ct, m_enc):
    import torch
    count = ct.shape[0]
    want_m, want_raw, want_ovf = he.decrypt(key, ct, raw=True)
    got_m = torch.full((count,), 0x5A5A5A5A, dtype=torch.int64, device="cuda")
    got_raw = torch.full((count, key.limbs), -1, dtype=torch.int32, device="cuda")
    got_ovf = torch.zeros(1, dtype=torch.int32, device="cuda")
    he.decrypt_noalloc(key, ct, got_m, got_raw, got_ovf)
    torch.cuda.synchronize()
    assert torch.equal(got_m, want_m)
    assert torch.equal(got_raw, want_raw)
    assert int(got_ovf.item()) == int(want_ovf.item())
    assert np.array_equal(got_m[:len(m_enc)].cpu().numpy(), m_enc)
    # without the optional outputs
    got_m2 = torch.zeros(count, dtype=torch.int64, device="cuda")
    he.decrypt_noalloc(key, ct, got_m2)
    torch.cuda.synchronize()
    assert torch.equal(got_m2, want_m)


def test_noalloc_decrypt_equals_decrypt_twice_shrinking(setup):
    he, key, n = setup
    for count, seed in ((20000, 11), (3001, 12)):
        say(f"he_decrypt_noalloc 2048-bit count={count}")
        ct, m_enc = _inputs(he, key, n, count, seed)
        _check_call(he, key, ct, m_enc)


def test_noalloc_decrypt_refuses_counts_beyond_its_scratch(setup):
    import torch
    he, key, _ = setup
    say("he_decrypt_noalloc size limit (host-side refusal)")
    limit = (1 << 22) // key.limbs
    ct = torch.zeros((1, 2 * key.limbs), dtype=torch.int32, device="cuda")
    m = torch.zeros(1, dtype=torch.int64, device="cuda")
    rc = he._decrypt_noalloc(key.handle, he._ptr(ct), limit + 1, he._ptr(m), None, None, None)
    assert rc == he.HE_ERR_ARG
    assert b"exceeds the maximum" in he._last_error()
