"""Seeded symmetric edge weights for a CSR graph.

Every undirected edge {u, v} gets one float32 weight, stored in both of its entries.
The weight is a function of (min(u, v), max(u, v), seed) through an integer hash, so
the same graph and seed give the same weights on any device and in any entry order."""
import torch

_M32 = 0xFFFFFFFF


def _mix32(x: torch.Tensor) -> torch.Tensor:
    # xor-shift / multiply finaliser on values in [0, 2^32) held in int64; every product
    # stays below 2^59, so no step overflows
    x = x ^ (x >> 16)
    x = (x * 0x45D9F3B) & _M32
    x = x ^ (x >> 16)
    x = (x * 0x45D9F3B) & _M32
    return x ^ (x >> 16)


def edge_weights(row_ptr, col_idx, seed: int, lo: float = 0.25, hi: float = 4.0, values=None) -> torch.Tensor:
    """float32 weight per stored entry, on the device of row_ptr.  Uniform in [lo, hi]
    (rounded to float32), or, with `values`, one of those values per edge."""
    rp = torch.as_tensor(row_ptr).to(torch.int64)
    ci = torch.as_tensor(col_idx).to(device=rp.device, dtype=torch.int64)
    n = rp.numel() - 1
    rows = torch.repeat_interleave(torch.arange(n, device=rp.device), rp[1:] - rp[:-1])
    a, b = torch.minimum(rows, ci), torch.maximum(rows, ci)
    s = _mix32(torch.tensor(seed & _M32, dtype=torch.int64, device=rp.device))
    h = _mix32((_mix32(a ^ s) ^ b) & _M32)
    if values is not None:
        vals = torch.tensor(list(values), dtype=torch.float32, device=rp.device)
        return vals[h % len(vals)].contiguous()
    u = (h.to(torch.float64) + 0.5) / 4294967296.0
    return (lo + (hi - lo) * u).to(torch.float32).contiguous()
