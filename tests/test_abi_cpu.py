"""CPU-side checks of the C ABI library: it loads, exports every function
the headers in include/ declare, and its host-side argument checks reject bad input
without touching a GPU.  The host bignum that derives the per-key constants is
checked through a small g++ harness against Python integer arithmetic."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADERS = [os.path.join(ROOT, "include", h) for h in sorted(os.listdir(os.path.join(ROOT, "include")))
           if h.endswith(".h")]
LIB = os.path.join(ROOT, "paper_2504_03909_amd", "libhe_mi355x.so")


def declared_functions():
    src = "".join(open(h).read() for h in HEADERS)
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(he_[a-z0-9_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        pytest.fail("libhe_mi355x.so is not built (run python -m paper_2504_03909_amd.build)")
    return ctypes.CDLL(LIB)


def test_header_declares_the_boundary():
    fns = declared_functions()
    for name in ("he_keygen", "he_key_import", "he_encrypt", "he_hist_aggregate", "he_decrypt",
                 "he_encode", "he_last_error"):
        assert name in fns


def test_library_exports_every_declared_symbol(lib):
    missing = [f for f in declared_functions() if not hasattr(lib, f)]
    assert not missing, missing


def test_binding_lists_every_declared_symbol():
    from paper_2504_03909_amd import ckks, he  # load the library, no GPU call
    assert sorted(he.EXPORTED + ckks.EXPORTED) == declared_functions()


def test_host_side_argument_errors(lib):
    # Rejections that happen before any device work.
    lib.he_keygen.argtypes = [ctypes.c_uint32, ctypes.c_uint64, ctypes.POINTER(ctypes.c_void_p)]
    lib.he_last_error.restype = ctypes.c_char_p
    h = ctypes.c_void_p()
    assert lib.he_keygen(1000, 1, ctypes.byref(h)) == -1
    assert b"1024 or 2048" in lib.he_last_error()
    assert lib.he_keygen(1024, 1, None) == -1
    lib.he_encrypt.argtypes = [ctypes.c_void_p] * 3 + [ctypes.c_void_p, ctypes.c_uint64, ctypes.c_uint64,
                                                       ctypes.c_void_p, ctypes.c_void_p]
    assert lib.he_encrypt(None, None, 0, None, 0, 0, None, None) == -1
    lib.he_decrypt.argtypes = [ctypes.c_void_p] * 7
    assert lib.he_decrypt(None, None, None, None, None, None, None) == -1
    lib.he_hist_subtract.argtypes = [ctypes.c_void_p] * 3 + [ctypes.c_uint64, ctypes.c_uint32] + [ctypes.c_void_p] * 3
    assert lib.he_hist_subtract(None, None, None, 1, 0, None, None, None) == -1
    lib.he_encrypt_obfuscated.argtypes = [ctypes.c_void_p] * 2 + [ctypes.c_uint64] + [ctypes.c_void_p] * 3
    assert lib.he_encrypt_obfuscated(None, None, 1, None, None, None) == -1
    lib.he_ckks_create.argtypes = [ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_void_p]
    lib.he_ckks_last_error.restype = ctypes.c_char_p
    h2 = ctypes.c_void_p()
    assert lib.he_ckks_create(9, 40, 1, ctypes.byref(h2)) == -1
    assert b"log_n" in lib.he_ckks_last_error()
    for small in (10, 11):  # below the security bounds for Q of about 2^90
        assert lib.he_ckks_create(small, 40, 1, ctypes.byref(h2)) == -1
    assert lib.he_ckks_create(15, 40, 1, ctypes.byref(h2)) == -1
    assert lib.he_ckks_create(14, 70, 1, ctypes.byref(h2)) == -1
    lib.he_ckks_encrypt.argtypes = [ctypes.c_void_p] * 2 + [ctypes.c_uint64] * 3 + [ctypes.c_void_p] * 2
    assert lib.he_ckks_encrypt(None, None, 1, 0, 0, None, None) == -1
    lib.he_probe_int_mul.argtypes = [ctypes.c_uint64, ctypes.c_uint32, ctypes.c_void_p, ctypes.c_void_p]
    assert lib.he_probe_int_mul(0, 0, None, None) == -1


def test_key_import_rejects_bad_primes(lib):
    import numpy as np
    lib.he_key_import.argtypes = [ctypes.c_uint32, ctypes.c_void_p, ctypes.c_void_p,
                                  ctypes.POINTER(ctypes.c_void_p)]
    h = ctypes.c_void_p()
    even = np.zeros(16, dtype=np.uint32)
    even[15] = 0xC0000000
    odd = even.copy()
    odd[0] = 1
    assert lib.he_key_import(1024, even.ctypes.data, odd.ctypes.data, ctypes.byref(h)) == -2  # even p
    assert lib.he_key_import(1024, odd.ctypes.data, odd.ctypes.data, ctypes.byref(h)) == -2   # p == q
    small = np.zeros(16, dtype=np.uint32)
    small[0] = 7
    assert lib.he_key_import(1024, small.ctypes.data, odd.ctypes.data, ctypes.byref(h)) == -2  # n too short


# ------------------------------------------------------------ host bignum
HARNESS = r"""
#include <cstdio>
#include <string>
#include "hostbn.hpp"
using namespace hebn;
static Limbs parse(const char *hex) {
  Limbs r; std::string s(hex); size_t n = s.size();
  for (size_t end = n; end > 0;) { size_t beg = end >= 8 ? end - 8 : 0;
    r.push_back((uint32_t)std::stoul(s.substr(beg, end - beg), nullptr, 16)); end = beg; }
  norm(r); return r;
}
static void out(const char *tag, const Limbs &x) {
  printf("%s ", tag); if (x.empty()) { printf("0\n"); return; }
  printf("%x", x.back()); for (size_t i = x.size() - 1; i-- > 0;) printf("%08x", x[i]); printf("\n");
}
int main(int argc, char **argv) {
  Limbs a = parse(argv[1]), b = parse(argv[2]), m = parse(argv[3]);
  Limbs q, r; divmod(a, b, &q, &r);
  out("mul", mul(a, b)); out("q", q); out("r", r);
  out("powmod", powmod(a, b, m)); out("inv", invmod(a, m)); out("gcd", gcd(a, b));
  out("inv2", inv_pow2(m, 1024)); printf("ninv %x\n", neg_inv32(m[0]));
  printf("prime %d\n", (int)is_probable_prime(m));
  out("cand", prime_candidate(5, 1, 3, 512));
  return 0;
}
"""


@pytest.fixture(scope="module")
def harness(tmp_path_factory):
    d = tmp_path_factory.mktemp("hostbn")
    src = d / "h.cpp"
    src.write_text(HARNESS)
    exe = d / "h"
    r = subprocess.run(["g++", "-O1", "-std=c++17", "-fsanitize=address,undefined",
                        f"-I{os.path.join(ROOT, 'paper_2504_03909_amd', 'csrc')}", str(src), "-o", str(exe)],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    return str(exe)


def run_harness(exe, a, b, m):
    r = subprocess.run([exe, format(a, "x"), format(b, "x"), format(m, "x")], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    return {k: int(v, 16) for k, v in (line.split() for line in r.stdout.split("\n") if line)}


@pytest.mark.parametrize("seed", range(6))
def test_host_bignum_against_python_ints(harness, seed):
    import random
    import math
    import oracle.paillier as P
    rng = random.Random(seed)
    m = rng.getrandbits(1024) | (1 << 1023) | 1  # odd modulus
    a = rng.getrandbits(rng.choice([64, 700, 2048, 4096])) % (m * m) or 3
    while math.gcd(a, m) != 1:
        a += 1
    b = rng.getrandbits(rng.choice([33, 512, 1023, 2000])) | 1
    got = run_harness(harness, a, b, m)
    assert got["mul"] == a * b
    assert got["q"] == a // b and got["r"] == a % b
    assert got["powmod"] == pow(a, b, m)
    assert got["inv"] == pow(a, -1, m)
    assert got["gcd"] == math.gcd(a, b)
    assert got["inv2"] == pow(m, -1, 1 << 1024)
    assert got["ninv"] == (-pow(m, -1, 1 << 32)) % (1 << 32)
    assert got["prime"] == int(P.is_probable_prime(m))
    assert got["cand"] == P.prime_candidate(5, 1, 3, 512)


def test_host_bignum_primes(harness):
    import oracle.paillier as P
    p, q = P.keygen(1024, 1)
    for x in (p, q, (1 << 521) - 1):
        assert run_harness(harness, 3, 5, x)["prime"] == 1
    assert run_harness(harness, 3, 5, p * q)["prime"] == 0
    assert run_harness(harness, 3, 5, 3215031751)["prime"] == 0


KEY_HARNESS = r"""
#include <cstdio>
#include <string>
#include "keysetup.hpp"
using namespace hebn;
static Limbs parse(const char *hex) {
  Limbs r; std::string s(hex); size_t n = s.size();
  for (size_t end = n; end > 0;) { size_t beg = end >= 8 ? end - 8 : 0;
    r.push_back((uint32_t)std::stoul(s.substr(beg, end - beg), nullptr, 16)); end = beg; }
  norm(r); return r;
}
static const hekey::Blob *B;
static void out(const char *tag, size_t off, size_t limbs) {
  printf("%s ", tag);
  for (size_t i = limbs; i-- > 0;) printf("%08x", B->words[off + i]);
  printf("\n");
}
static void sched(const char *t, const hekey::ExpOff &e) {
  printf("%s.ops ", t);
  for (int i = 0; i < e.nops; ++i) printf("%s%x", i ? "," : "", B->words[e.ops + i]);
  printf("\n");
}
static void mod(const char *t, const hekey::ModOff &m, size_t S) {
  std::string s(t);
  out((s + ".N").c_str(), m.N, S); out((s + ".R1").c_str(), m.R1, S); out((s + ".R2").c_str(), m.R2, S);
  out((s + ".R3").c_str(), m.R3, S); out((s + ".R4").c_str(), m.R4, S); printf("%s.ninv %x\n", t, m.ninv);
}
int main(int argc, char **argv) {
  uint32_t bits = std::stoul(argv[1]);
  Limbs p = parse(argv[2]), q = parse(argv[3]);
  hekey::KeyConsts k = hekey::derive(bits, mul(p, q), p, q, true);
  B = &k.blob;
  size_t L = bits / 32, SP = L / 2;
  mod("n", k.n, L); mod("n2", k.n2, 2 * L);
  out("e_n", k.e_n.e, L + 1); printf("e_n.nwin %x\n", k.e_n.nwin); sched("e_n", k.e_n);
  out("nR_n2", k.nR_n2, 2 * L); out("half", k.half, L);
  for (int w = 0; w < 2; ++w) {
    std::string s = w ? "q" : "p";
    const hekey::PrimeOff &o = k.pr[w];
    mod((s + ".P").c_str(), o.P, SP); mod((s + ".P2").c_str(), o.P2, 2 * SP);
    out((s + ".e_enc").c_str(), o.e_enc.e, SP + 1); printf("%s.e_enc.nwin %x\n", s.c_str(), o.e_enc.nwin);
    out((s + ".e_lift").c_str(), o.e_lift.e, SP + 1); out((s + ".e_dec").c_str(), o.e_dec.e, SP + 1);
    sched((s + ".e_enc").c_str(), o.e_enc); sched((s + ".e_lift").c_str(), o.e_lift);
    sched((s + ".e_dec").c_str(), o.e_dec);
    out((s + ".QR_P").c_str(), o.QR_P, SP); out((s + ".PR_P2").c_str(), o.PR_P2, 2 * SP);
    out((s + ".Pinv").c_str(), o.Pinv, SP); out((s + ".hR_P").c_str(), o.hR_P, SP);
  }
  out("Cq", k.Cq, L); out("q2R_n2", k.q2R_n2, 2 * L); out("qinv_p", k.qinv_p, SP); out("qR_n", k.qR_n, L);
  return 0;
}
"""


@pytest.mark.parametrize("bits,seed", [(1024, 1), (2048, 2)])
def test_key_constants_against_definitions(tmp_path, bits, seed):
    import oracle.paillier as P
    src = tmp_path / "k.cpp"
    src.write_text(KEY_HARNESS)
    exe = tmp_path / "k"
    r = subprocess.run(["g++", "-O1", "-std=c++17", "-fsanitize=address,undefined",
                        f"-I{os.path.join(ROOT, 'paper_2504_03909_amd', 'csrc')}", str(src), "-o", str(exe)],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    p, q = P.keygen(bits, seed)
    r = subprocess.run([str(exe), str(bits), format(p, "x"), format(q, "x")], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    c, ops = {}, {}
    for line in r.stdout.splitlines():
        a, b = line.split()
        if a.endswith(".ops"):
            ops[a[:-4]] = [int(x, 16) for x in b.split(",")]
        else:
            c[a] = int(b, 16)
    n, L = p * q, bits // 32
    n2, g = n * n, n + 1

    def check_mod(tag, N, S):
        R = 1 << (32 * S)
        assert c[tag + ".N"] == N
        for k in range(1, 5):
            assert c[f"{tag}.R{k}"] == pow(R, k, N)
        assert (c[tag + ".ninv"] * N) % (1 << 32) == (1 << 32) - 1

    check_mod("n", n, L)
    check_mod("n2", n2, 2 * L)
    assert c["e_n"] == n and c["e_n.nwin"] == -(-n.bit_length() // 5)
    assert c["nR_n2"] == n * (1 << (64 * L)) % n2
    assert c["half"] == (n + 1) // 2
    SP = L // 2
    for tag, A, Bq in (("p", p, q), ("q", q, p)):
        check_mod(tag + ".P", A, SP)
        check_mod(tag + ".P2", A * A, 2 * SP)
        assert c[tag + ".e_enc"] == Bq % (A - 1)
        assert c[tag + ".e_enc.nwin"] == -(-(Bq % (A - 1)).bit_length() // 5)
        assert c[tag + ".e_lift"] == A and c[tag + ".e_dec"] == A - 1
        assert c[tag + ".QR_P"] == Bq * (1 << (32 * SP)) % A
        assert c[tag + ".PR_P2"] == A * (1 << (64 * SP)) % (A * A)
        assert c[tag + ".Pinv"] * A % (1 << (32 * SP)) == 1
        h = pow((pow(g, A - 1, A * A) - 1) // A, -1, A)
        assert c[tag + ".hR_P"] == h * (1 << (32 * SP)) % A
    assert c["Cq"] == pow(q * q, -1, p * p) * (1 << (32 * L)) % (p * p)
    assert c["q2R_n2"] == q * q * (1 << (64 * L)) % n2
    assert c["qinv_p"] == pow(q, -1, p)
    assert c["qR_n"] == q * (1 << (32 * L)) % n
    # the sliding-window schedules rebuild their exponents, with windows of
    # at most 6 bits ending in a 1 bit and odd-power indices below 32
    for tag, e in [("e_n", n)] + [(f"{t}.{k}", v) for t, A, Bq in (("p", p, q), ("q", q, p))
                                  for k, v in (("e_enc", Bq % (A - 1)), ("e_lift", A), ("e_dec", A - 1))]:
        o = ops[tag]
        acc = 2 * (o[0] & 0xFF) + 1
        assert o[0] >> 8 == 0 and (o[0] & 0xFF) < 32
        for op in o[1:]:
            k, nsq = op & 0xFF, op >> 8
            assert nsq >= 1 and (k < 32 or k == 0xFF)
            acc = (acc << nsq) + (2 * k + 1 if k != 0xFF else 0)
        assert acc == e, tag
        mults = sum(1 for op in o[1:] if op & 0xFF != 0xFF)
        assert mults <= e.bit_length() // 6 + 1, (tag, mults)


# ------------------------------------------------- bucketing index logic
# The count and scatter kernels' per-sample decisions (hist_bucket.hpp) run
# here on the CPU, block by block as the kernels run them (blocks in a
# shuffled order, ranks inside a block in a shuffled order, as the atomics
# may hand them out), on buffers of exactly the sizes the library allocates
# (every access to the node list, the bin table and the permutation goes
# through new[]-allocated arrays under AddressSanitizer).  Rows past the
# resident count and bins past the job's count appear in the input; the
# harness checks that each run of the permutation holds exactly the valid
# samples of its bin, that no block reads the base of a bin it did not
# reserve, and reports the skipped count.
BUCKET_HARNESS = r"""
#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <random>
#include <vector>
#include "hist_bucket.hpp"
using namespace he;
int main(int argc, char **argv) {
  const uint64_t seed = std::strtoull(argv[1], nullptr, 10), n = std::strtoull(argv[2], nullptr, 10);
  const uint64_t rows = std::strtoull(argv[3], nullptr, 10);
  const uint32_t F = std::strtoul(argv[4], nullptr, 10), B = std::strtoul(argv[5], nullptr, 10);
  const uint32_t block = std::strtoul(argv[6], nullptr, 10);
  setvbuf(stdout, nullptr, _IONBF, 0);
  std::mt19937_64 rng(seed);
  uint32_t *idx = new uint32_t[n ? n : 1];
  const uint64_t ld = rows;
  uint8_t *bins = new uint8_t[F * ld ? F * ld : 1];
  for (uint64_t s = 0; s < n; ++s)  // about 1 in 16 rows out of range
    idx[s] = (uint32_t)(rng() % 16 == 0 ? rows + rng() % 1000 : (rows ? rng() % rows : rng() % 1000));
  for (uint64_t i = 0; i < F * ld; ++i)  // about 1 in 8 bins out of range
    bins[i] = (uint8_t)(rng() % 8 == 0 ? B + rng() % (256 - B + (B == 256)) : rng() % B);
  const uint32_t nblk = (uint32_t)((n + block - 1) / block);
  std::vector<uint32_t> counts(F * B, 0), offs(F * B), cursor(F * B);
  uint64_t nbad = 0;
  std::vector<uint64_t> order(F * (uint64_t)nblk);
  for (uint64_t i = 0; i < order.size(); ++i) order[i] = i;
  // count kernel
  std::shuffle(order.begin(), order.end(), rng);
  for (uint64_t local : order) {
    uint32_t f; uint64_t s0, s1;
    bucket_block(local, nblk, n, block, f, s0, s1);
    if (f >= F || s1 > n || s0 > s1) { printf("block out of range\n"); return 2; }
    std::vector<uint32_t> h(256, 0);
    for (uint64_t s = s0; s < s1; ++s) {
      uint32_t row, bin;
      if (bucket_sample(idx, bins + f * ld, rows, B, s, row, bin)) h.at(bin)++; else ++nbad;
    }
    for (uint32_t b = 0; b < B; ++b) counts[f * B + b] += h[b];
  }
  // scan kernel
  for (uint32_t f = 0; f < F; ++f) {
    uint32_t acc = 0;
    for (uint32_t b = 0; b < B; ++b) { offs[f * B + b] = cursor[f * B + b] = acc; acc += counts[f * B + b]; }
  }
  // scatter kernel
  uint32_t *perm = new uint32_t[F * n ? F * n : 1];
  std::vector<uint8_t> written(F * n, 0);
  std::shuffle(order.begin(), order.end(), rng);
  const uint32_t kPoison = 0xFFFFFFFFu;
  for (uint64_t local : order) {
    uint32_t f; uint64_t s0, s1;
    bucket_block(local, nblk, n, block, f, s0, s1);
    std::vector<uint64_t> ss;
    for (uint64_t s = s0; s < s1; ++s) ss.push_back(s);
    std::shuffle(ss.begin(), ss.end(), rng);  // atomics hand out ranks in any order
    std::vector<uint32_t> h(256, 0), base(256, kPoison);
    struct Item { uint32_t row, bin, rank; };
    std::vector<Item> items;
    for (uint64_t s : ss) {
      uint32_t row, bin;
      if (bucket_sample(idx, bins + f * ld, rows, B, s, row, bin)) items.push_back({row, bin, h.at(bin)++});
    }
    for (uint32_t b = 0; b < B; ++b)
      if (h[b]) { base[b] = cursor[f * B + b]; cursor[f * B + b] += h[b]; }
    uint32_t *pf = perm + (uint64_t)f * n;
    for (const Item &it : items) {
      if (base[it.bin] == kPoison) { printf("unreserved base read\n"); return 3; }
      const uint64_t slot = bucket_slot(base[it.bin], it.rank);
      if (slot >= offs[f * B + it.bin] + counts[f * B + it.bin]) { printf("slot past its run\n"); return 4; }
      pf[slot] = it.row;
      written[f * n + slot]++;
    }
  }
  // every run holds exactly its bin's valid samples (as a multiset)
  uint64_t valid = 0;
  for (uint32_t f = 0; f < F; ++f) {
    std::vector<std::vector<uint32_t>> want(B);
    for (uint64_t s = 0; s < n; ++s) {
      const uint32_t row = idx[s];
      if (row < rows && bins[f * ld + row] < B) want[bins[f * ld + row]].push_back(row);
    }
    for (uint32_t b = 0; b < B; ++b) {
      const uint32_t o = offs[f * B + b], c = counts[f * B + b];
      if (c != want[b].size()) { printf("count mismatch\n"); return 5; }
      std::vector<uint32_t> got(perm + (uint64_t)f * n + o, perm + (uint64_t)f * n + o + c);
      for (uint32_t k = 0; k < c; ++k) if (written[f * n + o + k] != 1) { printf("slot not written once\n"); return 6; }
      std::sort(got.begin(), got.end());
      std::sort(want[b].begin(), want[b].end());
      if (got != want[b]) { printf("run content mismatch\n"); return 7; }
      valid += c;
    }
  }
  printf("bad %llu valid %llu\n", (unsigned long long)nbad, (unsigned long long)valid);
  delete[] idx; delete[] bins; delete[] perm;
  return 0;
}
"""


@pytest.fixture(scope="module")
def bucket_harness(tmp_path_factory):
    d = tmp_path_factory.mktemp("bucket")
    src = d / "b.cpp"
    src.write_text(BUCKET_HARNESS)
    exe = d / "b"
    r = subprocess.run(["g++", "-O1", "-g", "-std=c++17", "-fsanitize=address,undefined",
                        "-fno-sanitize-recover=all",
                        f"-I{os.path.join(ROOT, 'paper_2504_03909_amd', 'csrc')}", str(src), "-o", str(exe)],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    return str(exe)


@pytest.mark.parametrize("seed,n,rows,F,B,block", [
    (1, 10000, 3000, 3, 17, 4096),     # ragged last block, bins past 17 in the table
    (2, 4096, 5000, 2, 256, 4096),     # exactly one block, every bin value valid except rows
    (3, 1, 1, 1, 1, 4096),             # one sample, one row, one bin
    (4, 0, 10, 2, 8, 4096),            # empty node
    (5, 20000, 50, 4, 64, 256),        # many blocks, heavy duplicates
    (6, 777, 0, 1, 16, 128),           # no resident rows: every sample skipped
])
def test_bucketing_index_logic_under_asan(bucket_harness, seed, n, rows, F, B, block):
    r = subprocess.run([bucket_harness, str(seed), str(n), str(rows), str(F), str(B), str(block)],
                       capture_output=True, text=True, env={**os.environ, "ASAN_OPTIONS": "detect_leaks=0"})
    assert r.returncode == 0, r.stdout + r.stderr
    bad, valid = (int(x) for x in r.stdout.split()[1::2])
    assert bad + valid == F * n
    if n and rows == 0:
        assert valid == 0
