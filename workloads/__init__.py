"""Seeded synthetic ABX workloads.

This module only draws random inputs: item lengths, attribute labels and
SSL-like feature frames.  It holds none of the ABX arithmetic (no distance,
no alignment, no scoring), so that the FP64 oracle under ``oracle/`` and the
HIP library can both consume the very same bytes without sharing any code
that computes a result.

The shapes follow the paper's benchmark task: triphone items described by an
ON label (the phone), BY context (previous / next phone) and a speaker that
is either BY or ACROSS (Background section; ZeroSpeech setting in the
library-comparison section).  The paper's LibriSpeech features are not
available, so Gaussian stand-ins are drawn instead:

    frame = centroid[label] + offset[speaker or group or item] + noise

Structure (labels, lengths) comes from numpy's Philox bit generator; the
feature values come from a ``torch.Generator`` on the device the features
are requested on (``cpu`` or ``cuda``).  Parity tests always hand the same
feature tensor to both sides, so the two streams never need to agree across
devices.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional, Sequence

import numpy as np
import torch


@dataclass
class Workload:
    """One ABX dataset + task specification."""

    name: str
    features: torch.Tensor          # [n_frames, dim], float32 or bfloat16
    offsets: np.ndarray             # int64 [n_items + 1], frame ranges per item
    attrs: np.ndarray               # int32 [n_items, n_attr], label-encoded
    attr_names: List[str]
    on: int
    by: List[int]
    across: List[int]
    levels: List[List[int]] = field(default_factory=list)
    seed: int = 0

    @property
    def n_items(self) -> int:
        return int(self.attrs.shape[0])

    @property
    def dim(self) -> int:
        return int(self.features.shape[1])

    @property
    def n_frames(self) -> int:
        return int(self.features.shape[0])

    @property
    def lengths(self) -> np.ndarray:
        return np.diff(self.offsets)

    def features_f32_host(self) -> np.ndarray:
        """Host float32 copy (bf16 widens exactly to fp32)."""
        return self.features.detach().to("cpu").float().contiguous().numpy()

    def subset_items(self, items: Sequence[int]) -> "Workload":
        """A new workload holding only ``items`` (in the given order)."""
        items = np.asarray(items, dtype=np.int64)
        lens = self.lengths[items]
        new_off = np.zeros(len(items) + 1, dtype=np.int64)
        np.cumsum(lens, out=new_off[1:])
        starts = self.offsets[items]
        idx = np.concatenate([np.arange(s, s + l) for s, l in zip(starts, lens)]) if len(items) else np.zeros(0, np.int64)
        feats = self.features[torch.as_tensor(idx, device=self.features.device)]
        return Workload(self.name + "-subset", feats.contiguous(), new_off,
                        self.attrs[items].copy(), list(self.attr_names),
                        self.on, list(self.by), list(self.across),
                        [list(l) for l in self.levels], self.seed)


# ----------------------------------------------------------------------------
# random helpers
# ----------------------------------------------------------------------------

def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.Philox(seed))


def _zipf_bounded(rng: np.random.Generator, s: float, lo: int, hi: int, size: int) -> np.ndarray:
    """Draw integers in [lo, hi] with P(n) proportional to n**-s."""
    support = np.arange(lo, hi + 1, dtype=np.float64)
    p = support ** (-s)
    p /= p.sum()
    return rng.choice(np.arange(lo, hi + 1), size=size, p=p).astype(np.int64)


def _zipf_labels(rng: np.random.Generator, s: float, k: int, size: int) -> np.ndarray:
    """Label ids 0..k-1 where label r-1 has probability proportional to r**-s."""
    return (_zipf_bounded(rng, s, 1, k, size) - 1).astype(np.int32)


def _lognormal_lengths(rng, median, sigma, lo, hi, size) -> np.ndarray:
    l = np.rint(np.exp(rng.normal(np.log(median), sigma, size=size)))
    return np.clip(l, lo, hi).astype(np.int64)


def _offsets(lengths: np.ndarray) -> np.ndarray:
    off = np.zeros(len(lengths) + 1, dtype=np.int64)
    np.cumsum(lengths, out=off[1:])
    return off


def _compose_features(lengths: np.ndarray, frame_terms, dim: int, noise_std: float,
                      seed: int, device: str, out_dtype: torch.dtype,
                      chunk_frames: int = 1 << 22) -> torch.Tensor:
    """frame = sum_k table_k[index_k(item)] + N(0, noise_std^2), drawn in chunks.

    ``frame_terms`` is a list of ``(table [n_rows, dim] torch tensor on device,
    per-item row index np.ndarray)``.
    """
    dev = torch.device(device)
    gen = torch.Generator(device=dev)
    gen.manual_seed(int(seed) * 1000003 + 17)
    n_frames = int(lengths.sum())
    out = torch.empty((n_frames, dim), dtype=out_dtype, device=dev)
    item_of_frame = np.repeat(np.arange(len(lengths), dtype=np.int64), lengths)
    for f0 in range(0, n_frames, chunk_frames):
        f1 = min(n_frames, f0 + chunk_frames)
        it = item_of_frame[f0:f1]
        x = torch.randn((f1 - f0, dim), generator=gen, device=dev, dtype=torch.float32)
        x.mul_(noise_std)
        for table, idx in frame_terms:
            rows = torch.as_tensor(idx[it], device=dev)
            x.add_(table.index_select(0, rows))
        out[f0:f1] = x.to(out_dtype)
    return out


def _table(n_rows: int, dim: int, std: float, seed: int, salt: int, device: str) -> torch.Tensor:
    dev = torch.device(device)
    gen = torch.Generator(device=dev)
    gen.manual_seed(int(seed) * 7919 + salt)
    return torch.randn((n_rows, dim), generator=gen, device=dev, dtype=torch.float32) * std


# ----------------------------------------------------------------------------
# the five workload families
# ----------------------------------------------------------------------------

def plain_c1(seed: int = 0, device: str = "cpu", dim: int = 64, n_labels: int = 20,
             items_per_label: int = 20, n_contexts: int = 4, centroid_std: float = 1.0) -> Workload:
    """400 items = 20 labels x 20 items, context = k mod 4, lengths U{3..12}, dim 64.

    Task: ON label BY context.  Frames = centroid N(0,1) + per-item offset
    N(0,0.3^2) + per-frame noise N(0,0.5^2).
    """
    rng = _rng(seed)
    n = n_labels * items_per_label
    label = np.repeat(np.arange(n_labels, dtype=np.int32), items_per_label)
    context = np.tile(np.arange(items_per_label, dtype=np.int32) % n_contexts, n_labels)
    lengths = rng.integers(3, 13, size=n).astype(np.int64)
    attrs = np.stack([label, context], axis=1).astype(np.int32)
    cent = _table(n_labels, dim, centroid_std, seed, 1, device)
    item_off = _table(n, dim, 0.3, seed, 2, device)
    feats = _compose_features(lengths, [(cent, label.astype(np.int64)),
                                        (item_off, np.arange(n, dtype=np.int64))],
                              dim, 0.5, seed, device, torch.float32)
    return Workload("plain-c1", feats, _offsets(lengths), attrs, ["label", "context"],
                    on=0, by=[1], across=[], levels=[[1]], seed=seed)


def within_c2(seed: int = 1, device: str = "cpu", n_items: int = 100_000, dim: int = 768,
              n_labels: int = 40, n_speakers: int = 40, dtype: torch.dtype = torch.float32,
              centroid_std: float = 1.0) -> Workload:
    """Triphone-like within-speaker task: ON label BY prev, next, speaker.

    label/prev/next ~ Zipf(1) over 40, speaker uniform over 40, lengths
    round(exp(N(ln 9, 0.45^2))) clipped to [5, 25]; centroid N(0,1) +
    speaker offset N(0,0.4^2) + frame noise N(0,0.6^2).
    """
    rng = _rng(seed)
    label = _zipf_labels(rng, 1.0, n_labels, n_items)
    prev = _zipf_labels(rng, 1.0, n_labels, n_items)
    nxt = _zipf_labels(rng, 1.0, n_labels, n_items)
    spk = rng.integers(0, n_speakers, size=n_items).astype(np.int32)
    lengths = _lognormal_lengths(rng, 9.0, 0.45, 5, 25, n_items)
    attrs = np.stack([label, prev, nxt, spk], axis=1).astype(np.int32)
    cent = _table(n_labels, dim, centroid_std, seed, 1, device)
    soff = _table(n_speakers, dim, 0.4, seed, 2, device)
    feats = _compose_features(lengths, [(cent, label.astype(np.int64)), (soff, spk.astype(np.int64))],
                              dim, 0.6, seed, device, dtype)
    return Workload("within-c2", feats, _offsets(lengths), attrs,
                    ["#phone", "prev-phone", "next-phone", "speaker"],
                    on=0, by=[1, 2, 3], across=[], levels=[[1, 2], [3]], seed=seed)


def across_c3(seed: int = 2, device: str = "cpu", n_items: int = 200_000, dim: int = 1024,
              n_labels: int = 40, n_speakers: int = 100, dtype: torch.dtype = torch.float32,
              centroid_std: float = 1.0) -> Workload:
    """ACROSS-speaker task: ON label BY prev, next ACROSS speaker.

    40 labels / prev / next Zipf(1), 100 speakers uniform, lengths
    round(exp(N(ln 9, 0.55^2))) clipped to [3, 40], dim 1024.
    """
    rng = _rng(seed)
    label = _zipf_labels(rng, 1.0, n_labels, n_items)
    prev = _zipf_labels(rng, 1.0, n_labels, n_items)
    nxt = _zipf_labels(rng, 1.0, n_labels, n_items)
    spk = rng.integers(0, n_speakers, size=n_items).astype(np.int32)
    lengths = _lognormal_lengths(rng, 9.0, 0.55, 3, 40, n_items)
    attrs = np.stack([label, prev, nxt, spk], axis=1).astype(np.int32)
    cent = _table(n_labels, dim, centroid_std, seed, 1, device)
    soff = _table(n_speakers, dim, 0.4, seed, 2, device)
    feats = _compose_features(lengths, [(cent, label.astype(np.int64)), (soff, spk.astype(np.int64))],
                              dim, 0.6, seed, device, dtype)
    return Workload("across-c3", feats, _offsets(lengths), attrs,
                    ["#phone", "prev-phone", "next-phone", "speaker"],
                    on=0, by=[1, 2], across=[3], levels=[[1, 2], [3]], seed=seed)


def batched_c4(seed: int = 3, device: str = "cpu", n_groups: int = 5000, dim: int = 512,
               n_centroids: int = 64, size_lo: int = 2, size_hi: int = 2000,
               len_lo: int = 1, len_hi: int = 60, dtype: torch.dtype = torch.bfloat16,
               centroid_std: float = 1.0) -> Workload:
    """Uneven BY groups: sizes Zipf(1.1) on [2, 2000], two labels per group,
    lengths U{1..60}, dim 512 stored as bf16.  Task: ON label BY group."""
    rng = _rng(seed)
    sizes = _zipf_bounded(rng, 1.1, size_lo, size_hi, n_groups)
    n_items = int(sizes.sum())
    group = np.repeat(np.arange(n_groups, dtype=np.int32), sizes)
    label = np.empty(n_items, dtype=np.int32)
    pos = 0
    for g, n in enumerate(sizes):
        l1, l2 = rng.choice(n_centroids, size=2, replace=False)
        h = (n + 1) // 2
        label[pos:pos + h] = l1
        label[pos + h:pos + n] = l2
        pos += n
    lengths = rng.integers(len_lo, len_hi + 1, size=n_items).astype(np.int64)
    attrs = np.stack([label, group], axis=1).astype(np.int32)
    cent = _table(n_centroids, dim, centroid_std, seed, 1, device)
    goff = _table(n_groups, dim, 0.4, seed, 2, device)
    feats = _compose_features(lengths, [(cent, label.astype(np.int64)), (goff, group.astype(np.int64))],
                              dim, 0.6, seed, device, dtype)
    return Workload("batched-c4", feats, _offsets(lengths), attrs, ["label", "group"],
                    on=0, by=[1], across=[], levels=[[1]], seed=seed)


def serving_job(job_id: int, seed: int = 4, device: str = "cpu", n_items: Optional[int] = None,
                dim: Optional[int] = None, across: Optional[bool] = None,
                n_lo: int = 1000, n_hi: int = 50_000, centroid_std: float = 1.0) -> Workload:
    """One job of the serving stream.

    n ~ round(exp(U(ln 1e3, ln 5e4))), dim uniform over {256,...,1280},
    within or across with p = 1/2, 40 labels Zipf(1), 16 contexts Zipf(1),
    20 speakers, lengths U{1..60}.
    """
    rng = _rng(seed * 100003 + job_id)
    n = int(np.rint(np.exp(rng.uniform(np.log(n_lo), np.log(n_hi))))) if n_items is None else int(n_items)
    d = int(rng.choice([256, 512, 768, 1024, 1280])) if dim is None else int(dim)
    acr = bool(rng.random() < 0.5) if across is None else bool(across)
    label = _zipf_labels(rng, 1.0, 40, n)
    ctx = _zipf_labels(rng, 1.0, 16, n)
    spk = rng.integers(0, 20, size=n).astype(np.int32)
    lengths = rng.integers(1, 61, size=n).astype(np.int64)
    attrs = np.stack([label, ctx, spk], axis=1).astype(np.int32)
    s = seed * 100003 + job_id
    cent = _table(40, d, centroid_std, s, 1, device)
    soff = _table(20, d, 0.4, s, 2, device)
    feats = _compose_features(lengths, [(cent, label.astype(np.int64)), (soff, spk.astype(np.int64))],
                              d, 0.6, s, device, torch.bfloat16)
    if acr:
        return Workload(f"serve-job{job_id}-across", feats, _offsets(lengths), attrs,
                        ["label", "context", "speaker"], on=0, by=[1], across=[2],
                        levels=[[1], [2]], seed=s)
    return Workload(f"serve-job{job_id}-within", feats, _offsets(lengths), attrs,
                    ["label", "context", "speaker"], on=0, by=[1, 2], across=[],
                    levels=[[1], [2]], seed=s)


def gaussians_2d(mu: float, n_per_class: int, seed: int, device: str = "cpu") -> Workload:
    """Two classes of one-frame items in 2-D: N(0, I) and N((mu, mu), I).

    The Background section's worked example (the two-Gaussian figure).
    """
    gen = torch.Generator(device=torch.device(device))
    gen.manual_seed(seed)
    x0 = torch.randn((n_per_class, 2), generator=gen, device=device, dtype=torch.float64)
    x1 = torch.randn((n_per_class, 2), generator=gen, device=device, dtype=torch.float64) + mu
    feats = torch.cat([x0, x1]).float()
    label = np.repeat(np.arange(2, dtype=np.int32), n_per_class)
    lengths = np.ones(2 * n_per_class, dtype=np.int64)
    return Workload(f"gauss-mu{mu}", feats, _offsets(lengths), label[:, None].copy(), ["class"],
                    on=0, by=[], across=[], levels=[], seed=seed)


CONFIGS = {
    "plain-c1": plain_c1,
    "within-c2": within_c2,
    "across-c3": across_c3,
    "batched-c4": batched_c4,
}
