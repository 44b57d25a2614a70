"""Shared helpers of the GPU parity tests (test code; not collected)."""
import numpy as np

M32 = 0xFFFFFFFF


def pair_keys_from_gpu(pairs_t, n_virtual_per_key=1):
    """(n, 2) int32 cuda tensor of (u, i) -> sorted numpy uint64 keys (u << 32) | i."""
    import torch
    if pairs_t.shape[0] == 0:
        return np.zeros(0, np.uint64)
    u = pairs_t[:, 0].to(torch.int64) & M32
    i = pairs_t[:, 1].to(torch.int64) & M32
    k = torch.sort((u << 32) | i).values
    return k.cpu().numpy().view(np.uint64)


def pair_keys_from_oracle(out, sel, n_samples=1):
    """oracle.accept_eyes(..., lists=True) result -> sorted uint64 keys."""
    off = out["offsets"]
    idx = out["idx"].astype(np.uint64)
    smp = out["sample"].astype(np.uint64)
    cnt = np.diff(off).astype(np.int64)
    j = np.repeat(np.asarray(sel, np.uint64), cnt)
    u = j * np.uint64(n_samples) + smp
    return np.sort((u << np.uint64(32)) | idx)


def select_pairs_of_eyes(pairs_t, sel, chunk=1 << 27):
    """Pairs (u, i) of the eyes u in sel, from a possibly huge tensor, as keys."""
    import torch
    dev = pairs_t.device
    sel_t = torch.as_tensor(np.asarray(sel, np.int64), device=dev)
    parts = []
    for s in range(0, pairs_t.shape[0], chunk):
        blk = pairs_t[s:s + chunk]
        u = blk[:, 0].to(torch.int64) & M32
        m = torch.isin(u, sel_t)
        if m.any():
            i = blk[:, 1].to(torch.int64) & M32
            parts.append((u[m] << 32) | i[m])
    if not parts:
        return np.zeros(0, np.uint64)
    k = torch.sort(torch.cat(parts)).values
    return k.cpu().numpy().view(np.uint64)


def per_eye_counts(pairs_t, n_eyes, chunk=1 << 27):
    import torch
    cnt = torch.zeros(n_eyes, dtype=torch.int64, device=pairs_t.device)
    for s in range(0, pairs_t.shape[0], chunk):
        u = pairs_t[s:s + chunk, 0].to(torch.int64) & M32
        cnt += torch.bincount(u, minlength=n_eyes)
    return cnt.cpu().numpy()


def _mix64(x):
    """A SplitMix64-style finaliser on int64 tensors (wrapping arithmetic)."""
    x = x ^ (x >> 30)
    x = x * -4658895280553007687      # 0xBF58476D1CE4E5B9 as a signed 64-bit value
    x = x ^ (x >> 27)
    x = x * -7723592293110705685      # 0x94D049BB133111EB
    return x ^ (x >> 31)


def per_eye_fingerprints(pairs_t, n_eyes, chunk=1 << 27):
    """Per-eye (count, sum of h1(i), sum of h2(i)) of a possibly huge (n, 2)
    pair tensor, in wrapping 64-bit arithmetic; two sets of pairs with equal
    fingerprints for every eye are equal unless two independent 64-bit sums
    collide."""
    import torch
    dev = pairs_t.device
    cnt = torch.zeros(n_eyes, dtype=torch.int64, device=dev)
    s1 = torch.zeros(n_eyes, dtype=torch.int64, device=dev)
    s2 = torch.zeros(n_eyes, dtype=torch.int64, device=dev)
    for s in range(0, pairs_t.shape[0], chunk):
        blk = pairs_t[s:s + chunk]
        u = blk[:, 0].to(torch.int64) & M32
        i = blk[:, 1].to(torch.int64) & M32
        cnt.index_add_(0, u, torch.ones_like(u))
        s1.index_add_(0, u, _mix64(i))
        s2.index_add_(0, u, _mix64(i ^ 0x5DEECE66D))
    return cnt.cpu().numpy(), s1.cpu().numpy(), s2.cpu().numpy()
