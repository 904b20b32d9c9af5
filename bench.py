"""Benchmark of the Paillier histogram path on one MI355X.

One step = one pass of the whole path over the 2048-bit, 100,000-sample
workload: fixed-point encoding of the 200,000 gradient values, encryption of
all of them (seeded r, CRT path), the root node's encrypted histogram over
32 features x 256 Zipf(1.1) bins, and CRT decryption of the 16,384 histogram
ciphertexts.  Inputs (gradients, bins, sample list, key) are resident in HBM
before timing starts.  Prints one JSON line, which also carries (after the
timed steps) the 64-job batched comparison ("batched": one job per launch
against graph replay of one persistent launch), the depth-6 tree over
1,000,000 samples ("tree": encryption, one job per launch and one graph per
level, decryption of every node), the served request loop ("served": a
2,000-request Poisson trace at 200 requests/s and a 1,000-request trace at
0.8x the measured capacity, continuous batching against FIFO, p50/p99
latency) and the CPU oracle baseline.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]
                    [--no-batched] [--no-served] [--no-tree] [--chunk C | --fixed-shapes]

--chunk C fixes the histogram's items (16 lanes, at most C samples per item);
--fixed-shapes skips both autotuners (the library's default histogram shape,
pinned exponentiation shapes) so that separate profiler passes run the same
kernels.

Other workloads (each prints its own JSON line; not the default):
    --workload tree      2048-bit, 1,000,000 samples, 64 x 256 Zipf bins, depth-6
                         tree: one job per launch vs one captured plan per level
    --workload batched   64 uneven node jobs over 200,000 resident samples:
                         one launch per job vs one batched launch vs graph replay
    --workload served    request loop (Poisson arrivals, two keys, four parties):
                         continuous batching vs FIFO one-request-per-launch
    --workload horizontal  secure horizontal round with CKKS: 5 clients encrypt
                         G and H vectors of 7,680 values, the server adds, clients
                         decrypt; plus batched encryption throughput
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

KEY_BITS, M, J, K = 2048, 100_000, 32, 256
KEY_SEED, R_SEED, DATA_SEED = 2, 2024, 1
# MI355X: 256 CUs x 64 lanes x 2.4 GHz, one 32x32->64 multiply-add
# (v_mad_u64_u32) per lane per clock.
PEAK_MUL32_PER_S = 256 * 64 * 2.4e9
MI355X_HBM_BPS = 8.0e12
# HBM-side bytes of one encryption launch (k_enc_r + k_pow mod p + k_pow lift
# + k_enc_crt_b over 200,000 ciphertexts), from rocprofv3 FETCH_SIZE and WRITE_SIZE passes
# scaled by a 256 MiB copy (profiles/enc_crt_2048_100k_counters.md), and the
# digest of the kernel sources those passes ran on (kernel_sources_digest()).
# The figure is reported only while the sources still have that digest.
ENC_LAUNCH_TRAFFIC = {"bytes": 4.0915e10, "sources_sha256_16": "0c8bbee5b0c6da4e"}
# the kernels and the host code that picks their launches and exponent schedules
KERNEL_SOURCES = ("he_kernels.hip", "he_internal.hpp", "hist_bucket.hpp", "mont.hpp", "mont29.hpp",
                  "radix29.hpp", "he_api.cpp", "keysetup.hpp")


def _code_only(text: str) -> str:
    """C++ source without its comments and with runs of white space collapsed,
    so that edits of comments or layout leave the digest unchanged."""
    out, i, n = [], 0, len(text)
    while i < n:
        c = text[i]
        if c in "\"'":
            j = i + 1
            while j < n and text[j] != c:
                j += 2 if text[j] == "\\" else 1
            out.append(text[i:j + 1])
            i = j + 1
        elif text.startswith("//", i):
            j = text.find("\n", i)
            i = n if j < 0 else j
        elif text.startswith("/*", i):
            j = text.find("*/", i + 2)
            i = n if j < 0 else j + 2
            out.append(" ")
        else:
            out.append(c)
            i += 1
    return " ".join("".join(out).split())


def kernel_sources_digest() -> str:
    """First 16 hex digits of the SHA-256 of the kernel sources (code only:
    comments and layout do not count) and the build flags they compile with
    (include paths relative to the repository, so the digest is the same
    wherever the tree is checked out)."""
    import hashlib
    from paper_2504_03909_amd import build as B
    h = hashlib.sha256()
    for name in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2504_03909_amd", "csrc", name), encoding="utf-8") as f:
            h.update(name.encode() + b"\0" + _code_only(f.read()).encode())
    h.update(" ".join(f.replace(ROOT, ".") for f in B.COMMON).encode())
    return h.hexdigest()[:16]


def mm_products(s: int) -> int:
    """32x32->64 products of one s-limb CIOS Montgomery product."""
    return 2 * s * s + s


def sq_products(s: int) -> int:
    """32x32->64 products of one s-limb Montgomery squaring: the s (s + 1) / 2
    distinct products a_i a_j of the square plus the s^2 + s of the reduction."""
    return s * (s + 1) // 2 + s * s + s


def nwin(e: int) -> int:
    return max(1, -(-e.bit_length() // 5))


def sliding_ops(e: int, width: int = 6):
    """(general products, squarings) of the sliding-window exponentiation by
    e: windows of up to `width` bits ending in a 1 bit, left to right, after
    a table of the 2^(width-1) odd powers (one squaring for x^2 and one
    product per further odd power)."""
    mults, sqs = 2 ** (width - 1) - 1, 1
    i, first = e.bit_length() - 1, True
    while i >= 0:
        if not (e >> i) & 1:
            sqs += 1
            i -= 1
            continue
        j = max(i - width + 1, 0)
        while not (e >> j) & 1:
            j += 1
        if not first:
            sqs += i - j + 1
            mults += 1
        first = False
        i = j - 1
    return mults, sqs


def modexp_products(e: int, s: int) -> int:
    """Products of one exponentiation mod an s-limb modulus as the kernels
    run it without constant-time table reads (sliding windows of up to 6
    bits): general products at 2s^2 + s, squarings at s(s+1)/2 + s^2 + s."""
    mults, sqs = sliding_ops(e)
    return mults * mm_products(s) + sqs * sq_products(s)


def crt_encrypt_products(p: int, q: int, L: int) -> int:
    """Products of the CRT encryption kernel (phase A) for one ciphertext."""
    sp = L // 2
    tot = 0
    for P, Q in ((p, q), (q, p)):
        # mod P: r reduction (3), exponentiation, from_mont, m Q (2)
        tot += (3 + 2) * mm_products(sp) + modexp_products(Q % (P - 1), sp)
        # mod P^2: to_mont, lift, (1 + m n), product
        tot += (1 + 2) * mm_products(2 * sp) + modexp_products(P, 2 * sp)
    return tot


def crt_decrypt_products(p: int, q: int, L: int) -> int:
    """Products of CRT decryption (both phases) for one ciphertext."""
    sp = L // 2
    tot = 0
    for P in (p, q):
        # c mod P^2 (2 MM + add), exponentiation, from_mont, exact division
        # (low-half product), m_P = k h_P
        tot += (2 + 1) * mm_products(2 * sp) + modexp_products(P - 1, 2 * sp) + sp * sp + mm_products(sp)
    return tot + 4 * mm_products(sp) + mm_products(L)


def hist_products(n_contrib: int, n_slots: int, rows: int, L: int) -> int:
    """Products of one canonical-input histogram call: conversion of every
    row, one product per contribution beyond the first of each slot, the
    combines, and the conversion out of Montgomery form (bounded above by
    one product per contribution plus two per slot)."""
    return (2 * rows + n_contrib + 2 * n_slots) * mm_products(2 * L)


def percentile(xs, q):
    xs = sorted(xs)
    if not xs:
        return None
    k = (len(xs) - 1) * q
    lo, hi = math.floor(k), math.ceil(k)
    return xs[lo] + (xs[hi] - xs[lo]) * (k - lo)


def host_cpu():
    """nproc and the CPU model of this host (Linux /proc/cpuinfo)."""
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return os.cpu_count(), model


def cpu_baseline(p: int, q: int, grads, bins, n_enc: int = 2000, n_feat: int = 16, n_dec: int = 512):
    """The oracle (Python ints, textbook Paillier: no CRT, no Montgomery) on
    the host's cores, on a bounded sample of the same workload, scaled to one
    full step: n_enc encryptions of seeded gradient values, the histograms
    of n_feat of the 32 features over all 100,000 samples (every product of
    those features), and n_dec decryptions of histogram ciphertexts."""
    import numpy as np
    import oracle.paillier as P
    from oracle import pool

    sk = P.PrivateKey(p, q)
    pk = sk.public
    cores = pool.workers()
    nproc, model = host_cpu()
    flat = grads.reshape(-1)
    rng = np.random.default_rng(0)
    pick = rng.choice(flat.size, size=n_enc, replace=False)
    ms = [P.encode(float(flat[i])) for i in pick]
    rs = [P.seeded_r(pk.n, KEY_BITS, R_SEED, int(i)) for i in pick]
    t0 = time.perf_counter()
    cts = pool.encrypt_many(pk, ms, rs, processes=cores)
    t_enc = (time.perf_counter() - t0) / n_enc
    # aggregation: n_feat whole features of the root node (M samples each,
    # g and h), sample i carrying the sampled ciphertext pair i mod n_enc/2
    rows = [(cts[2 * i], cts[2 * i + 1]) for i in range(n_enc // 2)]
    t0 = time.perf_counter()
    hists = pool.aggregate_features_cycled(pk, rows, M, [bins[f] for f in range(n_feat)], K, processes=cores)
    t_agg = time.perf_counter() - t0
    t_add = t_agg / (2 * M * n_feat)
    # decryption of n_dec of the histogram ciphertexts just formed
    hct = [c for h in hists for b in h for c in b][:n_dec]
    t0 = time.perf_counter()
    pool.decrypt_many(sk, hct, processes=cores)
    t_dec = (time.perf_counter() - t0) / len(hct)
    step = t_enc * 2 * M + t_add * 2 * M * J + t_dec * J * K * 2
    return {
        "value": round(2 * M / step, 3),
        "unit": "encryptions/s (whole pass)",
        "cores": cores,
        "kind": "oracle",
        "sample": (f"{n_enc} encryptions; the histograms of {n_feat} of the {J} features over all {M} samples "
                   f"({2 * M * n_feat} ciphertext products); {len(hct)} decryptions; on {cores} processes, "
                   f"extrapolated linearly to one pass of {2 * M} encryptions + {2 * M * J} products + "
                   f"{J * K * 2} decryptions"),
        "host": {"nproc": nproc, "cpu_model": model,
                 "processes_note": f"pool capped at {pool.MAX_WORKERS} processes, the host CPU share of one GPU"},
        "step_s": round(step, 1),
        "per_op_s": {"encrypt": t_enc, "product": t_add, "decrypt": t_dec},
        "stage_s": {"encrypt": round(t_enc * 2 * M, 1), "aggregate": round(t_add * 2 * M * J, 1),
                    "decrypt": round(t_dec * J * K * 2, 1)},
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--chunk", type=int, default=0)
    ap.add_argument("--fixed-shapes", action="store_true",
                    help="no autotuners: default histogram shape, pinned exponentiation shapes (profiler passes)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batched", action="store_true", help="leave the 64-job batched comparison out of the line")
    ap.add_argument("--no-served", action="store_true", help="leave the served request loop out of the line")
    ap.add_argument("--no-tree", action="store_true", help="leave the depth-6 tree (1,000,000 samples) out of the line")
    ap.add_argument("--workload", default="pass", choices=("pass", "tree", "batched", "served", "horizontal"))
    ap.add_argument("--requests", type=int, default=2000, help="requests of the served trace at --rate")
    ap.add_argument("--capacity-requests", type=int, default=1000,
                    help="requests of the served trace at 0.8x the measured capacity")
    ap.add_argument("--rate", type=float, default=200.0)
    ap.add_argument("--enc-slice", type=int, default=0,
                    help="served, continuous policy: encryptions longer than this go out as several launches "
                         "(0: one launch)")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="only run a plain device-to-device copy of MIB MiB (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}); the multi-GPU "
              "sharding of this path is a design note, not a measured configuration.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_2504_03909_amd import he
    from synth import workloads as W

    torch.cuda.set_device(0)
    if args.calibrate_copy:
        n = args.calibrate_copy << 18  # int32 elements
        src = torch.ones(n, dtype=torch.int32, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"calibration_copy_bytes": 4 * n}), flush=True)
        return
    if args.workload != "pass":
        line = {"tree": bench_tree, "batched": bench_batched, "served": bench_served,
                "horizontal": bench_horizontal}[args.workload](args)
        print(json.dumps(line), flush=True)
        return
    stream = torch.cuda.current_stream()
    key = he.Key.generate(KEY_BITS, KEY_SEED)
    n, p, q = key.export()
    L = key.limbs
    st = W.streams(DATA_SEED)
    grads_h = W.gradients(M, st[1])
    bins_h = W.bins_zipf(J, M, K, st[2])
    grads = torch.from_numpy(grads_h.reshape(-1)).cuda()
    bins = torch.from_numpy(bins_h).cuda()
    idx = torch.arange(M, dtype=torch.int32, device="cuda")
    ct = torch.empty((M, 2, 2 * L), dtype=torch.int32, device="cuda")
    hist = torch.empty((J, K, 2, 2 * L), dtype=torch.int32, device="cuda")
    job = he.Job(idx, bins, K, hist)

    def ev():
        return torch.cuda.Event(enable_timing=True)

    def step(marks):
        marks[0].record(stream)
        m = he.encode(grads)
        marks[1].record(stream)
        he.encrypt(key, m, seed=R_SEED, out=ct.view(-1, 2 * L))
        marks[2].record(stream)
        he.hist_aggregate(key, ct, [job], chunk=args.chunk)
        marks[3].record(stream)
        dm, _, ovf = he.decrypt(key, hist)
        marks[4].record(stream)
        return dm, ovf

    # Setup: one encryption of the gradients so the autotuner can pick the
    # histogram work shape for this shape class (used by every step below).
    he.encrypt(key, he.encode(grads), seed=R_SEED, out=ct.view(-1, 2 * L))
    if args.fixed_shapes:
        # no autotuner: the library's default histogram shape at this size
        # (8 lanes per ciphertext, items of up to 128 samples, two groups per
        # item) and pinned exponentiation shapes, so that every profiler pass
        # runs the same kernels
        hist_tune = he.HistTune(128, 2, 8, 0, None)
        exp_shapes = {}
        for kind, count, lanes, tail in (("mod_p", 2 * M, 2, 0), ("lift", 2 * M, 4, 0), ("decrypt", J * K * 2, 4, 0)):
            he.crt_set_shape(key, kind, count, lanes, 0, tail)
            exp_shapes[kind] = he.PowTune(lanes, 0, tail, 0.0)
    else:
        hist_tune = (he.hist_autotune(key, ct, [he.Job(idx, bins, K)]) if args.chunk == 0
                     else he.HistTune(args.chunk, 2, 16, 0, None))
        # launch shapes of the exponentiations (lanes per integer, waves per
        # SIMD, last round's launch) for 200,000 encryptions and 16,384
        # decryptions, tuned before timing
        exp_shapes = he.crt_autotune(key, 2 * M, J * K * 2)
    tuned_chunk, tuned_split = hist_tune.chunk, hist_tune.split
    for _ in range(args.warmup):
        step([ev() for _ in range(5)])
    torch.cuda.synchronize()
    all_marks = [[ev() for _ in range(5)] for _ in range(args.steps)]
    t0 = time.perf_counter()
    for mk in all_marks:
        dm, ovf = step(mk)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    stage_ms = {k: [] for k in ("encode", "encrypt", "aggregate", "decrypt", "step")}
    for mk in all_marks:
        stage_ms["encode"].append(mk[0].elapsed_time(mk[1]))
        stage_ms["encrypt"].append(mk[1].elapsed_time(mk[2]))
        stage_ms["aggregate"].append(mk[2].elapsed_time(mk[3]))
        stage_ms["decrypt"].append(mk[3].elapsed_time(mk[4]))
        stage_ms["step"].append(mk[0].elapsed_time(mk[4]))
    avg = {k: sum(v) / len(v) for k, v in stage_ms.items()}
    ms_step = wall * 1e3 / args.steps

    # self-check of the last step: decrypted histogram == exact plaintext sums
    mo = np.rint(grads_h * 2.0 ** 32).astype(np.int64)
    dmh = dm.cpu().numpy().reshape(J, K, 2)
    ok = int(ovf.item()) == 0
    for f in range(J):
        for t in range(2):
            ref = np.zeros(K, dtype=np.int64)
            np.add.at(ref, bins_h[f].astype(np.int64), mo[:, t])
            ok = ok and np.array_equal(ref, dmh[f, :, t])

    # Encryption split into an offline part (obfuscators r^n mod n^2, which do
    # not depend on the gradients) and an online part (three Montgomery
    # products per value).  Reported beside the step, not inside it.
    m_last = he.encode(grads)
    rho = he.obfuscators(key, 2 * M, seed=R_SEED)
    ct_obf = he.encrypt_obfuscated(key, m_last, rho)
    obf_marks = [ev() for _ in range(3)]
    obf_marks[0].record(stream)
    he.obfuscators(key, 2 * M, seed=R_SEED, out=rho)
    obf_marks[1].record(stream)
    he.encrypt_obfuscated(key, m_last, rho, out=ct_obf)
    obf_marks[2].record(stream)
    torch.cuda.synchronize()
    obf_same = bool(torch.equal(ct_obf, ct.view(-1, 2 * L)))
    t_off, t_on = obf_marks[0].elapsed_time(obf_marks[1]), obf_marks[1].elapsed_time(obf_marks[2])
    del rho, ct_obf
    # Beside the step: the public-key path, c = (1 + m n) r^n mod n^2 by one
    # exponentiation mod n^2 (what a holder of n alone runs), on the step's
    # first 50,000 values; bit-identical to the CRT path's ciphertexts.
    n_pub = 50_000
    pub = he.Key.public(KEY_BITS, n)
    ct_pub = he.encrypt(pub, m_last[:n_pub], seed=R_SEED)
    pub_marks = [ev() for _ in range(2)]
    pub_marks[0].record(stream)
    he.encrypt(pub, m_last[:n_pub], seed=R_SEED, out=ct_pub)
    pub_marks[1].record(stream)
    torch.cuda.synchronize()
    pub_same = bool(torch.equal(ct_pub, ct.view(-1, 2 * L)[:n_pub]))
    t_pub = pub_marks[0].elapsed_time(pub_marks[1])
    # x mod n^2 (2 products), into and out of the exponentiation's form (2),
    # the exponentiation by n, f = 1 + m n and the product with it (3)
    pub_products = modexp_products(n, 2 * L) + 7 * mm_products(2 * L)
    del ct_pub, pub
    # Beside the step: packed decryption of the same 16,384 histogram
    # ciphertexts (the passive party folds 4 per ciphertext).
    pk_marks = [ev() for _ in range(3)]
    packed, slots = he.pack(key, hist)
    he.decrypt_packed(key, packed, J * K * 2, slots)
    pk_marks[0].record(stream)
    packed, slots = he.pack(key, hist)
    pk_marks[1].record(stream)
    dm_packed, _ = he.decrypt_packed(key, packed, J * K * 2, slots)
    pk_marks[2].record(stream)
    torch.cuda.synchronize()
    packed_same = bool(torch.equal(dm_packed.view(dm.shape), dm))
    t_pack, t_dpk = pk_marks[0].elapsed_time(pk_marks[1]), pk_marks[1].elapsed_time(pk_marks[2])
    ms_packed_pass = ms_step - avg["decrypt"] + t_pack + t_dpk
    # Beside the step: the private-key exponentiations with window-table
    # reads independent of the secret exponent (every entry read, the
    # digit's entry kept by a mask), on the same inputs.
    ct_hard = torch.empty_like(ct)
    key.set_constant_time(True)
    he.encrypt(key, m_last, seed=R_SEED, out=ct_hard.view(-1, 2 * L))
    hard_marks = [ev() for _ in range(3)]
    hard_marks[0].record(stream)
    he.encrypt(key, m_last, seed=R_SEED, out=ct_hard.view(-1, 2 * L))
    hard_marks[1].record(stream)
    dm_hard, _, _ = he.decrypt(key, hist)
    hard_marks[2].record(stream)
    torch.cuda.synchronize()
    key.set_constant_time(False)
    hard_same = bool(torch.equal(ct_hard, ct)) and bool(torch.equal(dm_hard, dm))
    t_enc_hard, t_dec_hard = hard_marks[0].elapsed_time(hard_marks[1]), hard_marks[1].elapsed_time(hard_marks[2])
    del ct_hard, dm_hard
    # Multiply-rate probe: 8 multiply-add chains per lane on 2,048 blocks of
    # 256 threads, the measured counterpart of the derived peak.
    he.probe_int_mul(64, 2048)
    pr_marks = [ev(), ev()]
    pr_marks[0].record(stream)
    n_probe = he.probe_int_mul(4096, 2048)
    pr_marks[1].record(stream)
    torch.cuda.synchronize()
    probe_rate = n_probe / (pr_marks[0].elapsed_time(pr_marks[1]) / 1e3)

    digest = kernel_sources_digest()
    traffic_current = digest == ENC_LAUNCH_TRAFFIC["sources_sha256_16"]
    enc_products = crt_encrypt_products(p, q, L)
    achieved = 2 * M * enc_products / (avg["encrypt"] / 1e3)
    line = {
        "metric": "Paillier encryptions/s + encrypted hist sample-adds/s at 2048-bit key; p99 latency",
        "value": round(2 * M / (ms_step / 1e3), 1),
        "unit": "encryptions/s (whole pass: encode+encrypt+histogram+decrypt)",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic",
        "config": {
            "workload": "2048-bit key, 100000 samples, 32 features x 256 Zipf(1.1) bins, root node: "
                        "encode + encrypt 200000 + encrypted histogram + CRT decrypt 16384",
            "key_bits": KEY_BITS, "samples": M, "features": J, "bins": K, "r": "seeded",
            "encrypt_path": "crt", "hist_chunk": tuned_chunk, "hist_split": tuned_split,
            "hist_lanes": hist_tune.lanes, "hist_waves_per_simd": hist_tune.waves or "own occupancy",
            "hist_shape": ("library default, exponentiation shapes pinned" if args.fixed_shapes else
                           "autotuned before timing" if args.chunk == 0 else "given"),
            "exponentiation_shapes": {k: {"lanes": v.lanes, "waves_per_simd": v.waves or "own occupancy",
                                          "last_round_lanes": v.tail_lanes or "same launch",
                                          "tuning_ms": round(v.ms, 3)} for k, v in exp_shapes.items()},
        },
        "stages": {
            "encode_ms": round(avg["encode"], 3),
            "encrypt_ms": round(avg["encrypt"], 3),
            "aggregate_ms": round(avg["aggregate"], 3),
            "decrypt_ms": round(avg["decrypt"], 3),
            "encryptions_per_s": round(2 * M / (avg["encrypt"] / 1e3), 1),
            "sample_adds_per_s": round(2 * M * J / (avg["aggregate"] / 1e3), 1),
            "decryptions_per_s": round(J * K * 2 / (avg["decrypt"] / 1e3), 1),
        },
        "stage_alu_frac": {
            "encrypt": round(achieved / PEAK_MUL32_PER_S, 4),
            "aggregate": round(hist_products(2 * M * J, J * K * 2, M, L) / (avg["aggregate"] / 1e3)
                               / PEAK_MUL32_PER_S, 4),
            "decrypt": round(J * K * 2 * crt_decrypt_products(p, q, L) / (avg["decrypt"] / 1e3)
                             / PEAK_MUL32_PER_S, 4),
        },
        "step_latency_ms": {"p50": round(percentile(stage_ms["step"], 0.5), 3),
                            "p99": round(percentile(stage_ms["step"], 0.99), 3)},
        "roofline": {
            "kernel": "k_enc_r + k_pow (mod p) + k_pow (lift mod p^2) + k_enc_crt_b (CRT encryption)",
            "bound": "alu",
            "achieved": round(achieved / 1e12, 3),
            "peak": round(PEAK_MUL32_PER_S / 1e12, 3),
            "unit": "T mul32/s",
            "frac": round(achieved / PEAK_MUL32_PER_S, 4),
            "traffic": (ENC_LAUNCH_TRAFFIC["bytes"] if traffic_current else None),
            "traffic_sources_sha256_16": {"measured_on": ENC_LAUNCH_TRAFFIC["sources_sha256_16"],
                                          "this_build": digest},
            "probe_measured": round(probe_rate / 1e12, 3),
            "frac_of_probe": round(achieved / probe_rate, 4),
            "traffic_unit": "HBM bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
            "algorithmic_bytes_per_launch": 2 * M * (8 + 4 * 2 * L),
            "algorithmic_products_per_launch": 2 * M * enc_products,
            "products_per_ciphertext": enc_products,
        },
        "parity_self_check": bool(ok),
        "packed_decryption": {"slots": slots, "pack_ms": round(t_pack, 3), "decrypt_ms": round(t_dpk, 3),
                              "equals_decrypt": packed_same,
                              "pass_ms_with_it": round(ms_packed_pass, 3),
                              "pass_encryptions_per_s_with_it": round(2 * M / (ms_packed_pass / 1e3), 1)},
        "constant_time_tables": {
            "encrypt_ms": round(t_enc_hard, 3), "decrypt_ms": round(t_dec_hard, 3),
            "encrypt_over_default": round(t_enc_hard / avg["encrypt"], 4),
            "decrypt_over_default": round(t_dec_hard / avg["decrypt"], 4),
            "pass_ms_with_it": round(ms_step - avg["encrypt"] - avg["decrypt"] + t_enc_hard + t_dec_hard, 3),
            "equals_default": hard_same,
        },
        "obfuscated_encryption": {
            "offline_obfuscators_ms": round(t_off, 3),
            "online_encrypt_ms": round(t_on, 3),
            "online_encryptions_per_s": round(2 * M / (t_on / 1e3), 1),
            "equals_encrypt": obf_same,
        },
        "public_key_encryption": {
            "count": n_pub, "ms": round(t_pub, 3),
            "encryptions_per_s": round(n_pub / (t_pub / 1e3), 1),
            "products_per_encryption": pub_products,
            "alu_frac": round(n_pub * pub_products / (t_pub / 1e3) / PEAK_MUL32_PER_S, 4),
            "equals_crt_encrypt": pub_same,
        },
    }
    del ct, hist, job
    torch.cuda.empty_cache()
    if not args.no_batched:
        print("[bench] batched: 64 uneven node jobs", file=sys.stderr, flush=True)
        line["batched"] = bench_batched(args, compact=True)
    if not args.no_tree:
        print("[bench] tree: 1,000,000 samples, depth 6, one job per launch", file=sys.stderr, flush=True)
        line["tree"] = bench_tree(args, compact=True)
        torch.cuda.empty_cache()
    if not args.no_served:
        print(f"[bench] served: {args.requests} requests at {args.rate:g}/s", file=sys.stderr, flush=True)
        line["served"] = bench_served(args, compact=True)
    if not args.no_cpu_baseline:
        print("[bench] cpu baseline (oracle on the host cores)", file=sys.stderr, flush=True)
        line["cpu_baseline"] = cpu_baseline(p, q, grads_h, bins_h)
    print(json.dumps(line), flush=True)


def _timed(fn, label=""):
    import torch
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    out = fn()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    if label:
        print(f"[bench] {label}: {dt:.3f} s", file=sys.stderr, flush=True)
    return out, dt


def bench_tree(args, compact=False):
    """2048-bit key, 1,000,000 samples, 64 features x 256 Zipf(1.1) bins,
    depth-6 tree (63 nodes, seeded splits, direct aggregation of every node).
    compact: encryption, one job per launch and one graph per level, and the
    decryption of every node only (the default line's sub-object)."""
    import numpy as np
    import torch
    from paper_2504_03909_amd import he, pipeline
    from synth import workloads as W
    Mt, Jt, Kt, depth = 1_000_000, 64, 256, 6
    key = he.Key.generate(KEY_BITS, KEY_SEED)
    st = W.streams(3)
    g = torch.from_numpy(W.gradients(Mt, st[1])).cuda()
    bins = torch.from_numpy(W.bins_zipf(Jt, Mt, Kt, st[2])).cuda()
    levels = [[torch.from_numpy(n.view(np.int32)).cuda() for n in lvl] for lvl in W.tree_levels(Mt, depth, st[4])]
    pipeline.encrypt_gradients(key, g[:1000].contiguous(), R_SEED)  # warm-up
    res, t_enc = _timed(lambda: pipeline.encrypt_gradients(key, g, R_SEED), "tree encrypt")
    pipeline.aggregate_levels(res, levels[:1], bins, Kt, mode="per_node")  # warm-up / workspace
    run_plain, t_plain = _timed(lambda: pipeline.aggregate_levels(res, levels, bins, Kt, mode="per_node"), "tree per node")
    run_batched, t_batched = _timed(lambda: pipeline.aggregate_levels(res, levels, bins, Kt, mode="per_level"), "tree per level")
    plans = pipeline.aggregate_levels(res, levels, bins, Kt, mode="per_level_graph")
    torch.cuda.synchronize()
    _, t_graph = _timed(lambda: [p.launch() for p in plans.plans], "tree graphs")
    same = all(torch.equal(a, b) for la, lb in zip(run_plain.hists, plans.hists) for a, b in zip(la, lb))
    contrib = 2 * Jt * sum(int(n.numel()) for lvl in levels for n in lvl)
    n_dec = 63 * Jt * Kt * 2
    if compact:
        del plans
        _, t_dec = _timed(lambda: pipeline.decrypt_levels(key, run_plain), "tree decrypt")
        return {
            "workload": "2048-bit key, 1000000 samples, 64 features x 256 Zipf(1.1) bins, depth-6 tree "
                        "(63 nodes), direct aggregation of every node",
            "encrypt_s": round(t_enc, 3), "encryptions_per_s": round(2 * Mt / t_enc, 1),
            "aggregate_one_job_per_launch_s": round(t_plain, 3),
            "aggregate_per_level_graph_s": round(t_graph, 3),
            "sample_adds_per_s": {"one_job_per_launch": round(contrib / t_plain, 1),
                                  "graph": round(contrib / t_graph, 1)},
            "decrypt_s": round(t_dec, 3), "decryptions_per_s": round(n_dec / t_dec, 1),
            "graph_equals_one_job_per_launch": bool(same),
            "total_s_one_job_per_launch": round(t_enc + t_plain + t_dec, 3),
        }
    pipeline.aggregate_levels(res, levels[:2], bins, Kt, mode="sibling")  # warm-up
    run_sib, t_sib = _timed(lambda: pipeline.aggregate_levels(res, levels, bins, Kt, mode="sibling"),
                            "tree sibling")
    sib_same = all(torch.equal(a, b) for la, lb in zip(run_plain.hists, run_sib.hists) for a, b in zip(la, lb))
    # the subtraction alone, over the deepest level's 16 parents (524,288 ciphertexts)
    last = run_sib.hists[-2]
    par = torch.stack(last[:16])
    chl = torch.stack(run_sib.hists[-1][0:32:2])
    out = torch.empty_like(par)
    he.hist_subtract(key, par, chl, out=out)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    ev[0].record()
    he.hist_subtract(key, par, chl, out=out)
    ev[1].record()
    torch.cuda.synchronize()
    sub_ms = ev[0].elapsed_time(ev[1])
    n_sub = par.numel() // (2 * key.limbs)
    _, t_dec = _timed(lambda: pipeline.decrypt_levels(key, run_plain), "tree decrypt")
    # whole rounds: aggregation + decryption + split finding, three ways
    rounds, round_splits = {}, {}
    for mode, pk in ((None, False), ("encrypted", False), ("plain", False), ("plain", True)):
        rr, tr = _timed(lambda: pipeline.tree_round(res, key, levels, bins, Kt, sibling=mode, packed=pk),
                        f"tree round sibling={mode} packed={pk}")
        name = str(mode) + ("_packed" if pk else "")
        rounds[name] = round(tr, 3)
        round_splits[name] = rr.splits
        del rr
    rounds_same = all(torch.equal(a[k], b[k]) for m in ("encrypted", "plain", "plain_packed")
                      for a, b in zip(round_splits["None"], round_splits[m]) for k in a)
    # decryption of one node histogram (32,768 ciphertexts): plain vs packed
    h0 = run_plain.hists[0][0]
    he.decrypt(key, h0)
    _, t_dec1 = _timed(lambda: he.decrypt(key, h0))
    pk0, s0 = he.pack(key, h0)
    he.decrypt_packed(key, pk0, h0.numel() // h0.shape[-1], s0)
    _, t_pack1 = _timed(lambda: he.pack(key, h0))
    _, t_decp1 = _timed(lambda: he.decrypt_packed(key, pk0, h0.numel() // h0.shape[-1], s0))
    contrib_sib = 2 * Jt * (Mt + sum(min(int(lvl[i].numel()), int(lvl[i + 1].numel()))
                                     for lvl in levels[1:] for i in range(0, len(lvl), 2)))
    return {
        "metric": "Paillier encryptions/s + encrypted hist sample-adds/s at 2048-bit key",
        "workload": "2048-bit key, 1000000 samples, 64 features x 256 Zipf(1.1) bins, depth-6 tree "
                    "(63 nodes), direct aggregation of every node",
        "encrypt_s": round(t_enc, 3), "encryptions_per_s": round(2 * Mt / t_enc, 1),
        "aggregate_one_job_per_launch_s": round(t_plain, 3),
        "aggregate_per_level_batched_s": round(t_batched, 3),
        "aggregate_per_level_graph_s": round(t_graph, 3),
        "sample_adds_per_s_one_job_per_launch": round(contrib / t_plain, 1),
        "sample_adds_per_s_graph": round(contrib / t_graph, 1),
        "contributions": contrib,
        "decrypt_s": round(t_dec, 3), "decryptions_per_s": round(n_dec / t_dec, 1),
        "graph_equals_plain": bool(same),
        "aggregate_sibling_s": round(t_sib, 3),
        "sibling_contributions": contrib_sib,
        "sibling_equals_plain": bool(sib_same),
        "subtract_524288_ms": round(sub_ms, 3),
        "subtract_per_s": round(n_sub / (sub_ms / 1e3), 1),
        "round_s": {"direct": rounds["None"], "sibling_encrypted": rounds["encrypted"],
                    "sibling_plain": rounds["plain"], "sibling_plain_packed": rounds["plain_packed"]},
        "node_decrypt_32768_ms": {"plain": round(t_dec1 * 1e3, 3), "pack": round(t_pack1 * 1e3, 3),
                                  "decrypt_packed": round(t_decp1 * 1e3, 3), "slots": s0},
        "round_splits_identical": bool(rounds_same),
        "total_s_one_job_per_launch": round(t_enc + t_plain + t_dec, 3),
    }


def bench_batched(args, compact=False):
    """64 uneven tree-node jobs (|S| log-uniform in [1e3, 2e5], F in [8, 128],
    B in {16, 64, 256}) over 200,000 resident 2048-bit encrypted samples:
    one launch per job against one batched persistent launch (autotuned
    shape) replayed from a captured graph."""
    import numpy as np
    import torch
    from paper_2504_03909_amd import he
    from synth import workloads as W
    Mp = 200_000
    key = he.Key.generate(KEY_BITS, KEY_SEED)
    st = W.streams(4)
    m = he.encode(torch.from_numpy(W.gradients(Mp, st[1]).reshape(-1)).cuda())
    ctm = he.to_mont(key, he.encrypt(key, m, seed=R_SEED).view(Mp, 2, -1))
    tables = {b: torch.from_numpy(t).cuda() for b, t in W.bins_tables(Mp, 128, (16, 64, 256), st[2]).items()}
    shapes = W.batched_jobs(64, st[5], Mp)

    def jobs():
        return [he.Job(torch.from_numpy(sh["sample_idx"].view(np.int32)).cuda(),
                       tables[sh["n_bins"]][sh["f0"]:sh["f0"] + sh["n_features"]], sh["n_bins"]) for sh in shapes]
    contrib = sum(2 * sh["n_features"] * sh["sample_idx"].size for sh in shapes)
    ja = jobs()
    for j in ja[:2]:
        he.hist_aggregate(key, ctm, [j], form=he.HE_FORM_MONT, chunk=64)
    _, t_single = _timed(lambda: [he.hist_aggregate(key, ctm, [j], form=he.HE_FORM_MONT, chunk=64) for j in ja])
    jb = jobs()
    he.hist_aggregate(key, ctm, jb, form=he.HE_FORM_MONT, chunk=64)
    _, t_batch64 = _timed(lambda: he.hist_aggregate(key, ctm, jb, form=he.HE_FORM_MONT, chunk=64))
    tune = he.hist_autotune(key, ctm, jb, form=he.HE_FORM_MONT)
    chunk, split, tune_ms = tune.chunk, tune.split, tune.ms
    _, t_tuned = _timed(lambda: he.hist_aggregate(key, ctm, jb, form=he.HE_FORM_MONT))
    jc = jobs()
    plan = he.HistPlan(key, ctm, jc, form=he.HE_FORM_MONT)
    plan.launch()
    _, t_graph = _timed(lambda: plan.launch())
    same = all(torch.equal(a.hist, b.hist) and torch.equal(a.hist, c.hist) for a, b, c in zip(ja, jb, jc))
    # work counters at the tuned shape: products joining real partials vs executed
    L = key.limbs
    prod = contrib * (2 * (2 * L) ** 2 + 2 * L)
    if compact:
        return {
            "workload": "64 node jobs, |S| log-uniform [1e3, 2e5], F uniform [8, 128], B in {16, 64, 256}, "
                        "200000 resident samples, 2048-bit key",
            "contributions": contrib,
            "one_job_per_launch_ms": round(t_single * 1e3, 3),
            "graph_replay_ms": round(t_graph * 1e3, 3),
            "speedup_over_one_job_per_launch": round(t_single / t_graph, 3),
            "sample_adds_per_s": {"one_job_per_launch": round(contrib / t_single, 1),
                                  "graph_replay": round(contrib / t_graph, 1)},
            "alu_frac_graph_replay": round(prod / t_graph / PEAK_MUL32_PER_S, 4),
            "autotuned": {"chunk": chunk, "split": split, "lanes": tune.lanes,
                          "waves_per_simd": tune.waves or "own occupancy", "ms": round(tune_ms, 3)},
            "results_identical": bool(same),
        }
    _, cnt = he.hist_aggregate_counted(key, ctm, jobs(), form=he.HE_FORM_MONT, chunk=chunk, split=split,
                                       lanes=tune.lanes, waves=tune.waves)
    mm_real, mm_done, mm_conv = (int(x) for x in cnt.cpu().tolist())
    return {
        "metric": "encrypted hist sample-adds/s at 2048-bit key",
        "workload": "64 node jobs, |S| log-uniform [1e3, 2e5], F uniform [8, 128], B in {16, 64, 256}, "
                    "200000 resident samples",
        "contributions": contrib,
        "one_job_per_launch_ms": round(t_single * 1e3, 3),
        "batched_chunk64_ms": round(t_batch64 * 1e3, 3),
        "batched_autotuned_ms": round(t_tuned * 1e3, 3),
        "graph_replay_ms": round(t_graph * 1e3, 3),
        "autotuned": {"chunk": chunk, "split": split, "lanes": tune.lanes,
                      "waves_per_simd": tune.waves or "own occupancy", "ms": round(tune_ms, 3)},
        "sample_adds_per_s": {"one_job_per_launch": round(contrib / t_single, 1),
                              "graph_replay": round(contrib / t_graph, 1)},
        "alu_frac_graph_replay": round(prod / t_graph / PEAK_MUL32_PER_S, 4),
        "results_identical": bool(same),
        "montgomery_products": {"joining_real_partials": mm_real, "executed": mm_done,
                                "conversions_out": mm_conv,
                                "executed_over_needed": round(mm_done / max(1, mm_real + mm_conv), 4)},
    }


def bench_horizontal(args):
    """Secure horizontal round (CKKS, N = 2^14, three 30-bit primes, scale
    2^40): 5 clients each encode and encrypt a G and an H vector of 7,680
    values, the server adds the 5 ciphertexts of each, a client decrypts and
    decodes the two sums.  Then 1,000 vectors encrypted in one call."""
    import numpy as np
    import torch
    from paper_2504_03909_amd import ckks
    clients, length = 5, 7680
    ctx = ckks.Context(14, 40, KEY_SEED)
    rng = np.random.default_rng(DATA_SEED)
    G = rng.normal(0, 200, size=(clients, length))
    H = rng.uniform(0, 500, size=(clients, length))
    z = torch.from_numpy(np.concatenate([G, H])).cuda()
    stream = torch.cuda.current_stream()

    def round_(marks):
        marks[0].record(stream)
        pt = ctx.encode(z)
        marks[1].record(stream)
        ct = ctx.encrypt(pt, seed=R_SEED)
        marks[2].record(stream)
        acc = ct[[0, clients]].contiguous()
        for c in range(1, clients):
            acc = ctx.add(acc, ct[[c, clients + c]].contiguous())
        marks[3].record(stream)
        dec = ctx.decrypt(acc)
        marks[4].record(stream)
        out = ctx.decode(dec, length)
        marks[5].record(stream)
        return out

    ev = lambda: torch.cuda.Event(enable_timing=True)
    round_([ev() for _ in range(6)])
    torch.cuda.synchronize()
    runs = []
    for _ in range(max(1, args.steps)):
        mk = [ev() for _ in range(6)]
        out = round_(mk)
        torch.cuda.synchronize()
        runs.append([mk[i].elapsed_time(mk[i + 1]) for i in range(5)] + [mk[0].elapsed_time(mk[5])])
    st = np.median(np.array(runs), axis=0)
    err = float(np.abs(out.cpu().numpy() - np.stack([G.sum(0), H.sum(0)])).max())
    # throughput: 1,000 vectors in one call
    zb = torch.from_numpy(rng.normal(0, 200, size=(1000, length))).cuda()
    ptb = ctx.encode(zb)
    ctb = ctx.encrypt(ptb, seed=R_SEED + 1)
    _, t_enc = _timed(lambda: ctx.encrypt(ptb, seed=R_SEED + 1, out=ctb), "ckks encrypt 1000")
    _, t_code = _timed(lambda: ctx.encode(zb), "ckks encode 1000")
    _, t_dec = _timed(lambda: ctx.decode(ctx.decrypt(ctb), length), "ckks decrypt+decode 1000")
    return {
        "metric": "secure horizontal round time and CKKS vector encryptions/s",
        "workload": "CKKS N=16384, 3 x 30-bit primes, scale 2^40; 5 clients x (G, H) vectors of 7680 values",
        "round_ms": round(float(st[5]), 3),
        "stages_ms": {"encode_10": round(float(st[0]), 3), "encrypt_10": round(float(st[1]), 3),
                      "server_add_8": round(float(st[2]), 3), "decrypt_2": round(float(st[3]), 3),
                      "decode_2": round(float(st[4]), 3)},
        "max_abs_error": err,
        "batch_1000": {"encrypt_ms": round(t_enc * 1e3, 3), "encode_ms": round(t_code * 1e3, 3),
                       "decrypt_decode_ms": round(t_dec * 1e3, 3),
                       "vector_encryptions_per_s": round(1000 / t_enc, 1),
                       "values_encrypted_per_s": round(1000 * length / t_enc, 1)},
    }


def bench_served(args, compact=False):
    """Request loop: Poisson arrivals of encrypt (1k-100k samples),
    aggregate (one depth-6 tree node, F in [8, 128]) and decrypt (up to
    64 x 256 x 2 ciphertexts) requests from 4 passive parties; 90% under a
    2048-bit key (200,000 resident samples), 10% under a 1024-bit key
    (50,000); mix 10/45/45.  Continuous batching vs FIFO one request per
    launch, at the given rate and at 0.8x the measured capacity."""
    import numpy as np
    import torch
    from paper_2504_03909_amd import he, serve
    k2 = he.Key.generate(2048, KEY_SEED)
    k1 = he.Key.generate(1024, 1)
    rng = np.random.default_rng(5)
    setups = {"k2048": serve.make_setup(k2, 200_000, 6, 4, 128, rng, 11),
              "k1024": serve.make_setup(k1, 50_000, 6, 4, 64, rng, 12)}
    budget = 64 << 30
    share = {"k2048": 0.9, "k1024": 0.1}

    # one backend per policy for every run (the library keeps one workspace
    # per stream)
    backends = {"continuous": serve.backend_for(setups, n_streams=4, enc_slice=args.enc_slice),
                "fifo": serve.backend_for(setups, n_streams=1)}

    def run(rate, n, policy, seed):
        tr = serve.build_trace(np.random.default_rng(seed), n, rate, setups, share)
        st = serve.Server(backends[policy], budget, max_inflight=8, policy=policy).run(tr, time_limit=900)
        print(f"[bench] served rate={rate:g} n={n} {policy}: {st['makespan_s']} s, p99 {st['p99_ms']} ms",
              file=sys.stderr, flush=True)
        return st

    def brief(st):
        keep = ("requests", "completed", "makespan_s", "throughput_req_s", "p50_ms", "p99_ms", "launches")
        out = {k: st[k] for k in keep if k in st}
        out["by_kind_p99_ms"] = {k: v["p99_ms"] for k, v in st.get("by_kind", {}).items()}
        return out

    run(1000.0, 16, "continuous", 99)  # warm-up: kernels and first allocations
    out = {"metric": "p50/p99 request latency and throughput, 2048-bit (90%) + 1024-bit (10%) keys",
           "workload": f"Poisson arrivals, mix encrypt/aggregate/decrypt 10/45/45, 4 passive parties, "
                       "depth-6 trees over 200000 (2048-bit) and 50000 (1024-bit) resident encrypted "
                       "gradients, F up to 128, HBM budget 64 GiB; continuous batching (4 streams) against "
                       "FIFO one request per launch on the same trace"}
    cont = run(args.rate, args.requests, "continuous", 1)
    fifo = run(args.rate, args.requests, "fifo", 1)
    f = brief if compact else (lambda x: x)
    out[f"rate_{args.rate:g}"] = {"requests": args.requests, "continuous": f(cont), "fifo": f(fifo)}
    cap = cont["throughput_req_s"]
    r2 = round(0.8 * cap, 2)
    n2 = args.capacity_requests
    out["capacity_req_s"] = cap
    out[f"rate_{r2:g}_(0.8x_capacity)"] = {"requests": n2, "continuous": f(run(r2, n2, "continuous", 2)),
                                            "fifo": f(run(r2, n2, "fifo", 2))}
    return out


if __name__ == "__main__":
    main()
