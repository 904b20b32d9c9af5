"""GPU test of the serving loop: requests under two keys (2048 and 1024 bit)
from several parties arrive faster than they are served, are admitted by
memory footprint and batched into overlapping launches on several streams;
every request's result is bit-identical to the result of the same request
run alone."""
import sys

import numpy as np
import pytest

import oracle.paillier as P

pytestmark = pytest.mark.gpu


def test_served_results_equal_alone():
    import torch
    from paper_2504_03909_amd import he, serve
    print("[gpu-case] serve mix vs alone", flush=True)
    sys.stdout.flush()
    rng = np.random.default_rng(11)
    k2 = he.Key.from_primes(2048, *P.keygen(2048, 2))
    k1 = he.Key.from_primes(1024, *P.keygen(1024, 1))
    setups = {"k2048": serve.make_setup(k2, 6000, 4, 4, 24, rng, 5),
              "k1024": serve.make_setup(k1, 3000, 3, 4, 16, rng, 6)}
    trace = serve.build_trace(rng, 48, 2000.0, setups, {"k2048": 0.9, "k1024": 0.1},
                              enc_range=(100, 4000), max_decrypt=3000, feature_range=(4, 24))
    backend = serve.backend_for(setups, n_streams=4, enc_slice=1000)
    srv = serve.Server(backend, hbm_budget=2 << 30, max_inflight=6)
    stats = srv.run(trace, time_limit=300)
    torch.cuda.synchronize()
    assert stats["completed"] == len(trace)
    assert stats["launches"] < len(trace)            # some launches carried several requests
    assert {r.key_id for r in trace} == {"k2048", "k1024"}
    alone_backend = serve.backend_for(setups, n_streams=1)
    for r in trace:
        solo = serve.run_alone(alone_backend, serve.clone_request(r))
        torch.cuda.synchronize()
        if r.kind == "aggregate":
            assert len(solo) == len(r.result)
            for a, b in zip(solo, r.result):
                assert torch.equal(a, b), r.rid
        else:
            assert torch.equal(solo, r.result), (r.rid, r.kind)
    # one decrypt result against the oracle: it decrypts resident ciphertexts
    # of known plaintexts (the encoded gradients)
    d = next(r for r in trace if r.kind == "decrypt")
    st = setups[d.key_id]
    flat_ct = st["ct"].view(-1, st["ct"].shape[-1])
    start = (d.payload["ct"].data_ptr() - flat_ct.data_ptr()) // (4 * flat_ct.shape[-1])
    mh = st["m"].cpu().numpy()
    assert d.result.cpu().numpy().tolist() == mh[start:start + d.result.numel()].tolist()
