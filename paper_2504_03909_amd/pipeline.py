"""Tree-level orchestration of the encrypted-histogram path on one GPU.

The active party encrypts every sample's g and h once per boosting round and
the ciphertexts stay resident in device memory (canonical form for transfer,
Montgomery form for the histogram kernels) across all nodes of the tree; a
passive party builds one encrypted histogram per tree node (Sec. III-B) and
the active party decrypts them.  Every arithmetic step runs in the HIP library
(``he``); this module only arranges buffers and calls.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional, Sequence

import torch

from . import he


@dataclass
class Resident:
    """Encrypted gradients of one round, resident on the device."""
    key: he.Key
    ct: torch.Tensor    # int32 [M, 2, 2L], canonical (what would be sent)
    ctm: torch.Tensor   # int32 [M, 2, 2L], Montgomery form (what the kernels read)

    @property
    def rows(self) -> int:
        return self.ct.shape[0]


def encrypt_gradients(key: he.Key, grads: torch.Tensor, r_seed: int, frac_bits: int = 32,
                      stream=None) -> Resident:
    """grads: float64 [M, 2] on the device -> resident ciphertexts."""
    M = grads.shape[0]
    m = he.encode(grads.reshape(-1).contiguous(), frac_bits, stream=stream)
    ct = he.encrypt(key, m, seed=r_seed, stream=stream).view(M, 2, 2 * key.limbs)
    ctm = he.to_mont(key, ct, stream=stream)
    return Resident(key, ct, ctm)


def node_job(sample_idx: torch.Tensor, bins: torch.Tensor, n_bins: int) -> he.Job:
    return he.Job(sample_idx, bins, n_bins)


@dataclass
class TreeRun:
    hists: List[List[torch.Tensor]] = field(default_factory=list)   # [level][node]
    plans: List[he.HistPlan] = field(default_factory=list)


def aggregate_levels(res: Resident, levels: Sequence[Sequence[torch.Tensor]], bins: torch.Tensor,
                     n_bins: int, mode: str = "per_node", chunk: int = 0, stream=None) -> TreeRun:
    """Encrypted histograms of every node, level by level.

    mode "per_node": one he_hist_aggregate call (one job) per node -- the
    plain one-job-per-launch path.  mode "per_level": all nodes of a level in
    one batched call.  mode "per_level_graph": all nodes of a level in one
    captured plan, replayed with a single graph launch.  modes "sibling" and
    "sibling_graph": per level, only the smaller child of every parent is
    aggregated (batched, resp. as a captured plan) and the larger one is the
    parent's histogram divided by it (``he.hist_subtract``); the children of
    node i of one level are nodes 2i and 2i + 1 of the next."""
    if mode in ("sibling", "sibling_graph"):
        return _sibling_levels(res, levels, bins, n_bins, chunk, mode == "sibling_graph", stream)
    run = TreeRun()
    for lvl in levels:
        jobs = [node_job(idx, bins, n_bins) for idx in lvl]
        if mode == "per_node":
            for j in jobs:
                he.hist_aggregate(res.key, res.ctm, [j], form=he.HE_FORM_MONT, chunk=chunk, stream=stream)
        elif mode == "per_level":
            he.hist_aggregate(res.key, res.ctm, jobs, form=he.HE_FORM_MONT, chunk=chunk, stream=stream)
        elif mode == "per_level_graph":
            plan = he.HistPlan(res.key, res.ctm, jobs, form=he.HE_FORM_MONT, chunk=chunk)
            plan.launch(stream)
            run.plans.append(plan)
        else:
            raise ValueError(mode)
        run.hists.append([j.hist for j in jobs])
    return run


def decrypt_levels(key: he.Key, run: TreeRun, stream=None) -> List[List[torch.Tensor]]:
    """Signed int64 histograms [F, B, 2] of every node."""
    return [[he.decrypt(key, h, stream=stream)[0] for h in lvl] for lvl in run.hists]


def _sibling_levels(res: Resident, levels: Sequence[Sequence[torch.Tensor]], bins: torch.Tensor,
                    n_bins: int, chunk: int, graph: bool, stream) -> TreeRun:
    # Histograms of a level live in one buffer [slots, F, B, 2, 2L] whose
    # slots are ordered [smaller children of every parent slot..., larger
    # children...], so the next level's parents are one contiguous array
    # and the whole level's subtraction is one call.
    key = res.key
    F = bins.shape[0]
    shape = (F, n_bins, 2, 2 * key.limbs)
    run = TreeRun()

    def aggregate(jobs):
        if graph:
            plan = he.HistPlan(key, res.ctm, jobs, form=he.HE_FORM_MONT, chunk=chunk)
            plan.launch(stream)
            run.plans.append(plan)
        else:
            he.hist_aggregate(key, res.ctm, jobs, form=he.HE_FORM_MONT, chunk=chunk, stream=stream)

    buf = torch.empty((1, *shape), dtype=torch.int32, device=res.ctm.device)
    aggregate([he.Job(levels[0][0], bins, n_bins, hist=buf[0])])
    run.hists.append([buf[0]])
    slot_node = [0]
    for lvl in levels[1:]:
        P = len(slot_node)
        nxt = torch.empty((2, P, *shape), dtype=torch.int32, device=buf.device)
        node_hist: List[Optional[torch.Tensor]] = [None] * len(lvl)
        jobs, small, large = [], [], []
        for s, u in enumerate(slot_node):
            a, b = 2 * u, 2 * u + 1
            sm, lg = (a, b) if lvl[a].numel() <= lvl[b].numel() else (b, a)
            jobs.append(he.Job(lvl[sm], bins, n_bins, hist=nxt[0, s]))
            node_hist[sm], node_hist[lg] = nxt[0, s], nxt[1, s]
            small.append(sm)
            large.append(lg)
        aggregate(jobs)
        he.hist_subtract(key, buf, nxt[0], out=nxt[1], stream=stream)
        buf = nxt.view(2 * P, *shape)
        slot_node = small + large
        run.hists.append(node_hist)
    return run


@dataclass
class RoundResult:
    """Per level: the plaintext histograms int64 [nodes, F, B, 2] in node
    order, and the best split of every node (he.split_find's dict)."""
    plain: List[torch.Tensor] = field(default_factory=list)
    splits: List[dict] = field(default_factory=list)


def decrypt_hist(key: he.Key, sk: he.Key, enc: torch.Tensor, out: Optional[torch.Tensor] = None,
                 packed: bool = False, stream=None) -> torch.Tensor:
    """Signed sums of encrypted histograms enc int32 [..., 2L] -> int64 [...].
    packed: the holder of the ciphertexts folds them with he.pack (public
    key) and the key holder decrypts the packed ones."""
    if not packed:
        return he.decrypt(sk, enc, out=out, stream=stream)[0]
    shape = enc.shape[:-1]
    if out is None:
        out = torch.empty(shape, dtype=torch.int64, device=enc.device)
    pk, slots = he.pack(key, enc, stream=stream)
    he.decrypt_packed(sk, pk, out.numel(), slots, out=out.view(-1), stream=stream)
    return out


def tree_round(res: Resident, sk: he.Key, levels: Sequence[Sequence[torch.Tensor]], bins: torch.Tensor,
               n_bins: int, sibling: Optional[str] = None, lam: float = 1.0, gamma: float = 0.0,
               min_child_weight: float = 1.0, frac_bits: int = 32, chunk: int = 0, packed: bool = False,
               stream=None) -> RoundResult:
    """The histogram work of one tree, level by level: the passive party's
    aggregation, the active party's decryption and split finding.

    sibling=None: every node is aggregated and decrypted.
    sibling="encrypted": the smaller child of every parent is aggregated, the
      larger one is the parent's encrypted histogram divided by it; all are
      decrypted.
    sibling="plain": only the smaller children are aggregated and decrypted;
      the larger child's plaintext histogram is the parent's minus the
      smaller one's, formed inside the split finder.
    packed: the returned histograms are packed before decryption.
    The children of node i of one level are nodes 2i and 2i + 1 of the next."""
    key = res.key
    F = bins.shape[0]
    dev = res.ctm.device
    out = RoundResult()

    def split(hist, minus=None, derived=None):
        return he.split_find(hist, minus, frac_bits, lam, gamma, min_child_weight, derived=derived, stream=stream)

    def in_node_order(slot_vals, slot_node):
        order = torch.as_tensor(sorted(range(len(slot_node)), key=lambda s: slot_node[s]), device=dev)
        return {k: v.index_select(0, order) for k, v in slot_vals.items()} if isinstance(slot_vals, dict) \
            else slot_vals.index_select(0, order)

    if sibling is None:
        for lvl in levels:
            jobs = [he.Job(idx, bins, n_bins) for idx in lvl]
            he.hist_aggregate(key, res.ctm, jobs, form=he.HE_FORM_MONT, chunk=chunk, stream=stream)
            enc = torch.stack([j.hist for j in jobs])
            plain = decrypt_hist(key, sk, enc, packed=packed, stream=stream)
            out.plain.append(plain)
            out.splits.append(split(plain))
        return out
    if sibling not in ("encrypted", "plain"):
        raise ValueError(sibling)

    shape = (F, n_bins, 2)
    L2 = 2 * key.limbs
    # level buffers in slot order [smaller children..., larger children...]
    enc_prev = torch.empty((1, *shape, L2), dtype=torch.int32, device=dev)
    he.hist_aggregate(key, res.ctm, [he.Job(levels[0][0], bins, n_bins, hist=enc_prev[0])], form=he.HE_FORM_MONT,
                      chunk=chunk, stream=stream)
    plain_prev = decrypt_hist(key, sk, enc_prev, packed=packed, stream=stream)
    out.plain.append(plain_prev)
    out.splits.append(split(plain_prev))
    slot_node = [0]
    for lvl in levels[1:]:
        P = len(slot_node)
        enc = torch.empty((2 if sibling == "encrypted" else 1, P, *shape, L2), dtype=torch.int32, device=dev)
        jobs, small, large = [], [], []
        for s, u in enumerate(slot_node):
            a, b = 2 * u, 2 * u + 1
            sm, lg = (a, b) if lvl[a].numel() <= lvl[b].numel() else (b, a)
            jobs.append(he.Job(lvl[sm], bins, n_bins, hist=enc[0, s]))
            small.append(sm)
            large.append(lg)
        he.hist_aggregate(key, res.ctm, jobs, form=he.HE_FORM_MONT, chunk=chunk, stream=stream)
        plain = torch.empty((2, P, *shape), dtype=torch.int64, device=dev)
        if sibling == "encrypted":
            he.hist_subtract(key, enc_prev, enc[0], out=enc[1], stream=stream)
            decrypt_hist(key, sk, enc, out=plain, packed=packed, stream=stream)
            sp_small, sp_large = split(plain[0]), split(plain[1])
        else:
            decrypt_hist(key, sk, enc[0], out=plain[0], packed=packed, stream=stream)
            sp_small = split(plain[0])
            sp_large = split(plain_prev, minus=plain[0], derived=plain[1])
        slot_node = small + large
        slots = plain.view(2 * P, *shape)
        sp = {k: torch.cat([sp_small[k], sp_large[k]]) for k in sp_small}
        out.plain.append(in_node_order(slots, slot_node))
        out.splits.append(in_node_order(sp, slot_node))
        enc_prev = enc.view(-1, *shape, L2) if sibling == "encrypted" else None
        plain_prev = slots
    return out
