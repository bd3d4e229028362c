"""Helpers shared by the GPU parity tests (not collected as tests)."""
import numpy as np
import torch

import oracle
import pagegen


def require_gpu():
    import pytest
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def garbage_pad(words: np.ndarray, W: int, seed: int) -> np.ndarray:
    """Sets every pad bit and pad word of a (rows, stride) uint64 array to
    random values (they must be ignored on input)."""
    r = np.random.default_rng(seed)
    out = words.copy()
    nw = (W + 63) // 64
    if W % 64:
        keep = np.uint64((1 << (W % 64)) - 1)
        junk = r.integers(0, 2**63, out.shape[0], dtype=np.int64).astype(np.uint64) << np.uint64(1)
        out[:, nw - 1] = (out[:, nw - 1] & keep) | (junk & ~keep)
    if out.shape[1] > nw:
        out[:, nw:] = r.integers(0, 2**63, (out.shape[0], out.shape[1] - nw), dtype=np.int64).astype(np.uint64)
    return out


def expected_words(op, img, se, stride=None, method="brute"):
    f = oracle.apply if method == "brute" else oracle.sat_apply
    return oracle.pack(f(op, img, se), stride)


def rnd_img(seed, H, W, p=0.5):
    r = np.random.default_rng(seed)
    return (r.random((H, W)) < p).astype(np.uint8)


def blobs_img(seed, H, W, density=0.3):
    """Random rectangles plus noise: runs of many lengths."""
    r = np.random.default_rng(seed)
    img = np.zeros((H, W), np.uint8)
    n = max(1, int(density * H * W / 40))
    for _ in range(n):
        x, y = int(r.integers(0, W)), int(r.integers(0, H))
        w, h = int(r.integers(1, 24)), int(r.integers(1, 12))
        img[y:y + h, x:x + w] = 1
    noise = r.random((H, W)) < 0.02
    img ^= noise.astype(np.uint8)
    return img


__all__ = ["require_gpu", "garbage_pad", "expected_words", "rnd_img", "blobs_img", "pagegen", "oracle"]
