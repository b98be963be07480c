"""Seeded synthetic inputs for the Pi_MatMul workloads.

This module holds none of the protocol's arithmetic: only shapes, the
client's additive share X (uniform over Z_{2^l}, which is what an additive
share of any prompt looks like), the server's fixed-point weights
W = floor(w * 2^f) with w ~ N(0, 0.02) (BERT's initialiser width, standing in
for fine-tuned GLUE checkpoints that are not available here), and the 32-byte
party seeds.  Both the oracle tests and the GPU path take their inputs from
here.
"""
from __future__ import annotations

import hashlib
import math
from dataclasses import dataclass, field

import numpy as np

MASTER_SEED = 20230529


def seed(party: str, request: int) -> bytes:
    """32-byte ChaCha20 key of a party ("client" or "server") for a request id."""
    return hashlib.sha256(f"pimm-{party}:{int(request)}".encode()).digest()


def share(rng: np.random.Generator, n: int, r: int, ell: int) -> np.ndarray:
    """Client share X in Z_{2^ell}^{n x r}, uniform, uint64."""
    return rng.integers(0, 1 << ell, size=(n, r), dtype=np.uint64)


def weights(rng: np.random.Generator, r: int, m: int, frac_bits: int,
            std: float = 0.02) -> np.ndarray:
    """Server weights [r][m] (d_in x d_out): floor(N(0, std) * 2^f) as int64."""
    w = rng.normal(0.0, std, size=(r, m))
    return np.floor(w * (1 << frac_bits)).astype(np.int64)


@dataclass
class MatmulInput:
    X: np.ndarray  # [n][r] uint64 share
    W: np.ndarray  # [r][m] int64 fixed point
    ell: int
    frac_bits: int
    name: str = ""

    @property
    def shape(self):
        """(n, r, m) = (sequence length, d_in, d_out)."""
        return (self.X.shape[0], self.X.shape[1], self.W.shape[1])

    @property
    def useful_macs(self) -> int:
        n, r, m = self.shape
        return n * r * m


def single_matmul(seed_: int = MASTER_SEED) -> MatmulInput:
    """One product: X 16x64 in Z_{2^37}, W 64x64 with 12 fractional bits."""
    rng = np.random.default_rng(seed_)
    W = weights(rng, 64, 64, 12)
    X = share(rng, 16, 64, 37)
    return MatmulInput(X, W, 37, 12, "single 16x64x64")


BERT_BASE_SHAPES = [("qkv", 768, 2304), ("attn_out", 768, 768), ("ffn1", 768, 3072),
                    ("ffn2", 3072, 768)]
BERT_LARGE_SHAPES = [("qkv", 1024, 3072), ("attn_out", 1024, 1024), ("ffn1", 1024, 4096),
                     ("ffn2", 4096, 1024)]


def layer(shapes, seq: int, ell: int, frac_bits: int, seed_: int = MASTER_SEED,
          layer_index: int = 0) -> list[MatmulInput]:
    """The linear products of one encoder layer at sequence length seq."""
    rng = np.random.default_rng([seed_, layer_index, seq])
    out = []
    for name, r, m in shapes:
        W = weights(rng, r, m, frac_bits)
        X = share(rng, seq, r, ell)
        out.append(MatmulInput(X, W, ell, frac_bits, f"{name} {seq}x{r}x{m}"))
    return out


def bert_base_layer(seq: int = 128, seed_: int = MASTER_SEED) -> list[MatmulInput]:
    """BERT-base-shaped layer: QKV 768x2304, attn-out 768x768, FFN 768x3072 and 3072x768;
    t = 2^37, 12 fractional bits."""
    return layer(BERT_BASE_SHAPES, seq, 37, 12, seed_)


def bert_large_layer(seq: int = 512, seed_: int = MASTER_SEED,
                     layer_index: int = 0) -> list[MatmulInput]:
    """BERT-large / GPT-2-medium-shaped layer: QKV 1024x3072, attn-out 1024x1024,
    FFN 1024x4096 and 4096x1024; t = 2^41, 14 fractional bits."""
    return layer(BERT_LARGE_SHAPES, seq, 41, 14, seed_, layer_index)


@dataclass
class BatchItem:
    shape_index: int
    seq: int
    X: np.ndarray


def batched_uneven(count: int = 64, seed_: int = MASTER_SEED, lo: int = 16, hi: int = 512):
    """Independent products of uneven length: seq ~ U{lo..hi}, shape uniform over the four
    BERT-base shapes; one weight matrix per shape shared by the items.
    Returns (weights per shape [(r, m, W)], items)."""
    rng = np.random.default_rng([seed_, 4])
    ws = [(r, m, weights(rng, r, m, 12)) for _, r, m in BERT_BASE_SHAPES]
    items = []
    for _ in range(count):
        si = int(rng.integers(0, len(ws)))
        seq = int(rng.integers(lo, hi + 1))
        items.append(BatchItem(si, seq, share(rng, seq, ws[si][0], 37)))
    return ws, items


@dataclass
class Request:
    rid: int
    arrival_s: float
    seq: int


def poisson_trace(rate_per_s: float, count: int, seed_: int = MASTER_SEED, lo: int = 32,
                  hi: int = 512) -> list[Request]:
    """Poisson arrivals (exponential gaps) with prompt length floor(exp(U[ln lo, ln hi]))."""
    rng = np.random.default_rng([seed_, 5, int(rate_per_s * 1000)])
    t = 0.0
    out = []
    for i in range(count):
        t += float(rng.exponential(1.0 / rate_per_s))
        seq = int(math.floor(math.exp(rng.uniform(math.log(lo), math.log(hi)))))
        out.append(Request(i, t, max(lo, min(hi, seq))))
    return out
