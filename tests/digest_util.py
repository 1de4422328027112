"""Slice and block digests of a product held in device memory, computed with
plain torch integer operations (test code: the checker of the full-output
parity test, not part of the product).

The definition is the oracle's (oracle.digest / oracle.block_digests): entry
t (0-based, ascending ids) of a slice, with id j and value bits v, adds
mix64(mix64((t << 32) | j) ^ v) to the slice digest, modulo 2^64; a block of
slices sums mix64(h_i ^ mix64((i << 32) | nnz_i)) over its slices i.  mix64
is SplitMix64's output function.  Here every 64-bit quantity is a torch
int64 whose bits are the uint64's: additions and products wrap modulo 2^64,
and the right shifts are made logical by masking the sign extension.
"""
import numpy as np

M1 = 0xBF58476D1CE4E5B9
M2 = 0x94D049BB133111EB


def _s64(x: int) -> int:
    """The int64 with the bits of the uint64 x."""
    return x - (1 << 64) if x >= (1 << 63) else x


def _shr(z, k: int):
    return (z >> k) & ((1 << (64 - k)) - 1)


def mix64(z):
    """SplitMix64's output function on an int64 tensor (bits as uint64)."""
    z = (z ^ _shr(z, 30)) * _s64(M1)
    z = (z ^ _shr(z, 27)) * _s64(M2)
    return z ^ _shr(z, 31)


def value_bits(val, n: int, device):
    """The values' bytes zero-extended to 64 bits; pattern only (val None) is
    the boolean true."""
    import torch
    if val is None:
        return torch.ones(n, dtype=torch.int64, device=device)
    if val.dtype == torch.uint8:
        return val.to(torch.int64)
    if val.dtype in (torch.int32, torch.float32):
        return val.view(torch.int32).to(torch.int64) & 0xFFFFFFFF
    if val.dtype in (torch.int64, torch.float64):
        return val.view(torch.int64)
    raise TypeError(val.dtype)


def slice_digests(ptr, idx, val, r0: int, r1: int):
    """(nnz, hash) int64 tensors of slices [r0, r1) of a device result."""
    import torch
    dev = idx.device
    lo, hi = int(ptr[r0]), int(ptr[r1])
    counts = ptr[r0 + 1:r1 + 1] - ptr[r0:r1]
    h = torch.zeros(r1 - r0, dtype=torch.int64, device=dev)
    if hi > lo:
        slot = torch.repeat_interleave(torch.arange(r1 - r0, device=dev), counts)
        t = torch.arange(lo, hi, device=dev, dtype=torch.int64) - ptr[r0:r1][slot]
        x = (t << 32) | idx[lo:hi].to(torch.int64)
        e = mix64(mix64(x) ^ value_bits(None if val is None else val[lo:hi], hi - lo, dev))
        h.index_add_(0, slot, e)
    return counts, h


def block_digests(ptr, idx, val, nslices: int, block: int = 1024, max_entries: int = 1 << 27):
    """Block digests (nnz, hash) as numpy int64/uint64 of every block of
    `block` slices, for a result whose slices are [0, nslices), processed a
    range of whole blocks at a time (at most about max_entries entries)."""
    import torch
    ptr_h = ptr.cpu().numpy()
    nb = -(-nslices // block)
    bn = np.zeros(nb, np.int64)
    bh = np.zeros(nb, np.uint64)
    b = 0
    while b < nb:
        e = b + 1
        while e < nb and ptr_h[min(nslices, (e + 1) * block)] - ptr_h[b * block] <= max_entries:
            e += 1
        r0, r1 = b * block, min(nslices, e * block)
        cnt, h = slice_digests(ptr, idx, val, r0, r1)
        i = torch.arange(r0, r1, device=h.device, dtype=torch.int64)
        r = mix64(h ^ mix64((i << 32) | cnt))
        pad = (e - b) * block - (r1 - r0)
        if pad:
            r = torch.cat([r, torch.zeros(pad, dtype=torch.int64, device=r.device)])
            cnt = torch.cat([cnt, torch.zeros(pad, dtype=torch.int64, device=cnt.device)])
        bh[b:e] = r.view(e - b, block).sum(dim=1).cpu().numpy().view(np.uint64)
        bn[b:e] = cnt.view(e - b, block).sum(dim=1).cpu().numpy()
        b = e
    return bn, bh
