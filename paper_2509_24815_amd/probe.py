"""Learned block probe: training-sample collection and training on the GPU.

The probe (an addition to the method, not in the paper) is a 5 -> 64 -> 1
ReLU MLP whose logit decides which blocks of a cut list are evaluated when
the list's traversal starts with a full heap (see include/seismic.h).  This
module drives the library's kernels: a plain search with list tracing, exact
top-k for the labels, seismic_probe_collect for the samples, then
seismic_probe_grad / seismic_probe_adam for each mini-batch.  Torch only
holds device memory and draws the sample order.
"""
from __future__ import annotations

import numpy as np

from . import binding

WORDS = binding.PROBE_WORDS
H, IN = 64, 5
N_USED = H * IN + 2 * H + 1


def init_params(seed: int = 0) -> np.ndarray:
    """fp32 master parameters: W1 uniform in +-1/sqrt(5), b1 = 0.1 (units
    start active on the non-negative features), w2 uniform in +-1/8, b2 = 0."""
    rng = np.random.default_rng(seed)
    p = np.zeros(WORDS, dtype=np.float32)
    p[:H * IN] = rng.uniform(-1, 1, H * IN) / np.sqrt(IN)
    p[H * IN:H * IN + H] = 0.1
    p[H * IN + H:H * IN + 2 * H] = rng.uniform(-1, 1, H) / 8
    return p


def bf16_bits(x: np.ndarray) -> np.ndarray:
    """fp32 -> bf16 bit patterns, nearest, ties to even."""
    u = np.asarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    return ((u + 0x7FFF + ((u >> 16) & 1)) >> 16).astype(np.uint16)


def save(path: str, weights) -> None:
    w = weights.cpu().numpy() if hasattr(weights, "cpu") else np.asarray(weights)
    np.save(path, w.view(np.uint16).reshape(WORDS))


def load(path: str) -> np.ndarray:
    w = np.load(path, allow_pickle=False)
    if w.dtype != np.uint16 or w.size != WORDS:
        raise ValueError(f"{path}: expected {WORDS} uint16 words")
    return w


def to_device(weights, device=None):
    """bf16 bit patterns (numpy uint16, or a torch tensor as train() returns
    it) as an int16 device tensor."""
    import torch
    if isinstance(weights, torch.Tensor):
        return weights.to(device or "cuda").view(torch.int16).contiguous()
    return torch.from_numpy(np.ascontiguousarray(weights).view(np.int16).copy()).to(device or "cuda")


def collect(index, qcsr, n_queries: int, k: int, cut: int, heap_factor: float, exact_k: int = 10, stream=None):
    """Samples of one batch of device-resident queries: a plain search
    (query_cut cut, heap_factor) traces every cut list's start, exact top-k
    gives the labels.  Returns (feat [slots, 8] int16, label [slots] uint8,
    sample indices int32) on the device."""
    import torch
    _, _, _, _, hmin, term = index.search(qcsr, k, cut, heap_factor, trace=True, prefix_stride=cut, stream=stream)
    e_ids, _ = index.exact(qcsr, exact_k, stream=stream)
    mb = index.info()["max_blocks_per_list"]
    slots = n_queries * cut * mb
    feat = torch.empty((slots, 8), dtype=torch.int16, device=hmin.device)
    label = torch.empty(slots, dtype=torch.uint8, device=hmin.device)
    binding.seismic_probe_collect(index.handle, qcsr, term, hmin, cut, e_ids, exact_k, mb, feat, label, stream)
    idx = torch.nonzero(label != 255).flatten().to(torch.int32)
    return feat, label, idx


def train(feat, label, idx, epochs: int = 4, batch: int = 8192, lr: float = 3e-3, pos_weight: float | None = None,
          neg_weight: float = 1.0, neg_weight_per_doc: float = 0.0, seed: int = 0, log=None):
    """Adam on the weighted cross-entropy.  Returns (bf16 weights as an int16
    device tensor, per-epoch mean loss)."""
    import torch
    dev = feat.device
    n = int(idx.numel())
    if n == 0:
        raise ValueError("no training samples")
    if pos_weight is None:
        pos = int((label[idx.long()] == 1).sum())
        pos_weight = (n - pos) / max(pos, 1)
    trainer = binding.seismic_probe_trainer_create(dev.index or 0, batch)
    try:
        master = torch.from_numpy(init_params(seed)).to(dev)
        m = torch.zeros(WORDS, dtype=torch.float32, device=dev)
        v = torch.zeros(WORDS, dtype=torch.float32, device=dev)
        weights = torch.from_numpy(bf16_bits(master.cpu().numpy()).view(np.int16).copy()).to(dev)
        grad = torch.empty(WORDS, dtype=torch.float32, device=dev)
        stats = torch.empty(4, dtype=torch.float32, device=dev)
        tot = torch.zeros(4, dtype=torch.float64, device=dev)
        gen = torch.Generator(device=dev)
        gen.manual_seed(seed)
        history = []
        step = 0
        for ep in range(epochs):
            order = idx[torch.randperm(n, generator=gen, device=dev)].contiguous()
            tot.zero_()
            for s0 in range(0, n, batch):
                nb = min(batch, n - s0)
                binding.seismic_probe_grad(trainer, feat, label, order[s0:s0 + nb], nb, weights, grad, stats,
                                           pos_weight, neg_weight, neg_weight_per_doc)
                step += 1
                binding.seismic_probe_adam(grad, stats, master, m, v, step, weights, lr=lr)
                tot += stats.double()
            t = tot.cpu().numpy()
            history.append(float(t[0] / max(t[3], 1e-30)))
            if log:
                log(f"[probe] epoch {ep + 1}/{epochs}: weighted loss {history[-1]:.5f} over {int(t[1])} samples "
                    f"({int(t[2])} positive), pos_weight {pos_weight:.2f}")
        return weights, history
    finally:
        binding.seismic_probe_trainer_free(trainer)
