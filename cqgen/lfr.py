"""LFR-style benchmark graphs (Lancichinetti-Fortunato-Radicchi recipe), seeded.

Recipe (written from the published LFR method, simplified where noted):

1. Degrees k_u are drawn from a continuous power law p(k) ~ k^-gamma on
   [k_min, k_max], rounded to integers; k_min is solved so that the continuous
   mean equals the requested average degree.
2. Community sizes s_c are drawn from p(s) ~ s^-beta on [s_min, s_max] until they
   cover n nodes; the last size is trimmed so the sizes sum to n.
3. Every node wants an internal degree k_in = round((1 - mu) k).  Nodes whose k_in
   does not fit the smallest community are placed first, each in a community that
   can hold it (sampled in proportion to size); the others fill the remaining
   places at random.  k_in is finally capped at |c| - 1.
4. Internal stubs are paired at random inside each community (configuration
   model); external stubs (k - k_in per node) are paired at random across the
   whole graph.  Self-loops, multi-edges and external pairs that fall inside one
   community are dropped (the original program rewires them; this recipe drops
   them, so realised degrees are slightly below the drawn ones).
5. Node ids are random with respect to communities (assignment is a random
   permutation), so the CSR has no locality to exploit.

All sampling uses torch random generators on the requested device, so a given
(params, seed, device type) always yields the same graph.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import torch


@dataclass(frozen=True)
class LFRParams:
    n: int
    avg_degree: float
    max_degree: int
    gamma: float = 2.0
    beta: float = 1.0
    min_comm: int = 20
    max_comm: int = 100
    mu: float = 0.3


# Workload shapes: the paper's LFR settings (degree exponent 2, community-size
# exponent 1, mixing 0.3) at the sizes used for parity tests and measurement.
CONFIGS = {
    "tiny_1k": LFRParams(1_000, 15, 50, 2.0, 1.0, 20, 100, 0.3),
    "m100k_mu0.1": LFRParams(100_000, 20, 100, 2.0, 1.0, 20, 1_000, 0.1),
    "m100k_mu0.3": LFRParams(100_000, 20, 100, 2.0, 1.0, 20, 1_000, 0.3),
    "m100k_mu0.5": LFRParams(100_000, 20, 100, 2.0, 1.0, 20, 1_000, 0.5),
    "l10m": LFRParams(10_000_000, 20, 1_000, 2.0, 1.0, 50, 5_000, 0.3),
    "s100m": LFRParams(100_000_000, 10, 1_000, 2.0, 1.0, 50, 10_000, 0.3),
}


@dataclass
class LFRGraph:
    n: int
    row_ptr: torch.Tensor      # int32 [n+1]
    col_idx: torch.Tensor      # int32 [2m], rows sorted ascending
    labels: torch.Tensor       # int32 [n], ground-truth communities in [0, num_labels)
    num_labels: int
    params: LFRParams
    seed: int
    stats: dict = field(default_factory=dict)

    @property
    def nnz(self) -> int:
        return int(self.col_idx.numel())


def _powerlaw_mean(xmin: float, xmax: float, expo: float) -> float:
    if abs(expo - 1.0) < 1e-12:
        return (xmax - xmin) / math.log(xmax / xmin)
    if abs(expo - 2.0) < 1e-12:
        return math.log(xmax / xmin) / (1.0 / xmin - 1.0 / xmax)
    a, b = 1.0 - expo, 2.0 - expo
    return (a / b) * (xmax ** b - xmin ** b) / (xmax ** a - xmin ** a)


def solve_kmin(avg: float, kmax: float, gamma: float) -> float:
    lo, hi = 1e-3, float(kmax)
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if _powerlaw_mean(mid, kmax, gamma) < avg:
            lo = mid
        else:
            hi = mid
    return 0.5 * (lo + hi)


def _powerlaw_sample(u: torch.Tensor, xmin: float, xmax: float, expo: float) -> torch.Tensor:
    if abs(expo - 1.0) < 1e-12:
        return xmin * torch.pow(torch.tensor(xmax / xmin, dtype=u.dtype, device=u.device), u)
    a = 1.0 - expo
    lo, hi = xmin ** a, xmax ** a
    return torch.pow(lo + u * (hi - lo), 1.0 / a)


def _randint(gen, high: int, size: int, device) -> torch.Tensor:
    return torch.randint(0, high, (size,), generator=gen, device=device, dtype=torch.int64)


def lfr_graph(params: LFRParams, seed: int, device: str | torch.device = "cpu") -> LFRGraph:
    device = torch.device(device)
    gen = torch.Generator(device=device)
    gen.manual_seed(int(seed))
    n = int(params.n)
    f64 = torch.float64

    # 1. degrees
    kmin = solve_kmin(params.avg_degree, params.max_degree, params.gamma)
    u = torch.rand(n, generator=gen, device=device, dtype=f64)
    k = torch.round(_powerlaw_sample(u, kmin, float(params.max_degree), params.gamma)).to(torch.int64)
    k = k.clamp_(1, params.max_degree)

    # 2. community sizes summing to n
    mean_s = _powerlaw_mean(params.min_comm, params.max_comm, params.beta)
    parts = []
    total = 0
    while total < n:
        batch = max(16, int(1.2 * (n - total) / mean_s) + 16)
        us = torch.rand(batch, generator=gen, device=device, dtype=f64)
        s = torch.round(_powerlaw_sample(us, params.min_comm, params.max_comm, params.beta)).to(torch.int64)
        parts.append(s)
        total += int(s.sum())
    sizes = torch.cat(parts)
    cs = torch.cumsum(sizes, 0)
    K = int(torch.searchsorted(cs, torch.tensor(n, device=device)).item()) + 1
    sizes = sizes[:K].clone()
    sizes[K - 1] = n - (int(cs[K - 2]) if K >= 2 else 0)
    if K >= 2 and int(sizes[K - 1]) < params.min_comm:
        sizes[K - 2] += sizes[K - 1]
        sizes = sizes[: K - 1]
        K -= 1

    # 3. assignment
    kin_want = torch.round((1.0 - params.mu) * k.to(f64)).to(torch.int64)
    labels = torch.full((n,), -1, dtype=torch.int64, device=device)
    order_c = torch.argsort(sizes)                      # communities by size ascending
    sorted_sizes = sizes[order_c]
    cum = torch.cumsum(sorted_sizes, 0).to(f64)
    big = torch.nonzero(kin_want + 1 > params.min_comm).flatten()
    if big.numel() > 0:
        need = kin_want[big] + 1
        first = torch.searchsorted(sorted_sizes, need)          # first eligible index
        first = first.clamp_(max=K - 1)
        base = torch.where(first > 0, cum[(first - 1).clamp(min=0)], torch.zeros_like(cum[first]))
        r = base + torch.rand(big.numel(), generator=gen, device=device, dtype=f64) * (cum[-1] - base)
        idx = torch.searchsorted(cum, r, right=True).clamp_(max=K - 1)
        idx = torch.maximum(idx, first)
        labels[big] = order_c[idx]
    used = torch.bincount(labels[labels >= 0], minlength=K)
    cap = (sizes - used).clamp(min=0)
    rest = torch.nonzero(labels < 0).flatten()
    slots = torch.repeat_interleave(torch.arange(K, device=device), cap)
    if slots.numel() < rest.numel():
        extra = _randint(gen, n, rest.numel() - slots.numel(), device)
        # extra places go to the community of a random node's slot (proportional to size)
        owner = torch.repeat_interleave(torch.arange(K, device=device), sizes)
        slots = torch.cat([slots, owner[extra]])
    slots = slots[torch.randperm(slots.numel(), generator=gen, device=device)[: rest.numel()]]
    labels[rest] = slots
    real_sizes = torch.bincount(labels, minlength=K)
    kin = torch.minimum(kin_want, real_sizes[labels] - 1).clamp_(min=0)
    kout = k - kin

    # 4a. internal wiring inside each community
    stubs = torch.repeat_interleave(torch.arange(n, device=device), kin)
    key = labels[stubs] * (1 << 31) + _randint(gen, 1 << 31, stubs.numel(), device)
    stubs = stubs[torch.argsort(key)]
    del key
    if stubs.numel() % 2:
        stubs = stubs[:-1]
    a, b = stubs[0::2], stubs[1::2]
    keep = (labels[a] == labels[b]) & (a != b)
    ia, ib = a[keep], b[keep]
    del stubs, a, b, keep

    # 4b. external wiring across the graph
    stubs = torch.repeat_interleave(torch.arange(n, device=device), kout)
    stubs = stubs[torch.randperm(stubs.numel(), generator=gen, device=device)]
    if stubs.numel() % 2:
        stubs = stubs[:-1]
    a, b = stubs[0::2], stubs[1::2]
    keep = (labels[a] != labels[b]) & (a != b)
    ea, eb = a[keep], b[keep]
    del stubs, a, b, keep

    src = torch.cat([ia, ea])
    dst = torch.cat([ib, eb])
    del ia, ib, ea, eb
    lo = torch.minimum(src, dst)
    hi = torch.maximum(src, dst)
    und = torch.unique(lo * n + hi)                    # simple graph: no multi-edges
    del src, dst, lo, hi
    lo = und // n
    hi = und % n
    del und
    row_ptr, col_idx = _csr_sym(n, lo, hi)
    graph = LFRGraph(n, row_ptr, col_idx, labels.to(torch.int32), K, params, int(seed))
    deg = (row_ptr[1:] - row_ptr[:-1])
    graph.stats = {
        "n": n,
        "nnz": int(col_idx.numel()),
        "m": int(col_idx.numel()) // 2,
        "avg_degree": float(col_idx.numel()) / n,
        "max_degree": int(deg.max()),
        "communities": K,
        "min_comm": int(real_sizes.min()),
        "max_comm": int(real_sizes.max()),
        "k_min_solved": kmin,
    }
    return graph


def _csr_sym(n: int, lo: torch.Tensor, hi: torch.Tensor):
    """Symmetric CSR (both directions of every undirected edge), rows sorted."""
    src = torch.cat([lo, hi])
    dst = torch.cat([hi, lo])
    key = torch.sort(src * n + dst).values
    del src, dst
    rows = key // n
    col = (key % n).to(torch.int32)
    counts = torch.bincount(rows, minlength=n)
    row_ptr = torch.zeros(n + 1, dtype=torch.int64, device=key.device)
    row_ptr[1:] = torch.cumsum(counts, 0)
    return row_ptr.to(torch.int32), col


def perturb_labels(labels: torch.Tensor, num_labels: int, frac: float, seed: int) -> torch.Tensor:
    """Move exactly round(frac * n) distinct nodes to a uniformly random other community."""
    device = labels.device
    gen = torch.Generator(device=device)
    gen.manual_seed(int(seed))
    n = labels.numel()
    cnt = int(round(frac * n))
    out = labels.clone().to(torch.int64)
    if cnt == 0 or num_labels < 2:
        return out.to(torch.int32)
    who = torch.randperm(n, generator=gen, device=device)[:cnt]
    r = torch.randint(0, num_labels - 1, (cnt,), generator=gen, device=device, dtype=torch.int64)
    old = out[who]
    out[who] = torch.where(r >= old, r + 1, r)
    return out.to(torch.int32)


def random_labels(n: int, num_labels: int, seed: int, device="cpu") -> torch.Tensor:
    gen = torch.Generator(device=torch.device(device))
    gen.manual_seed(int(seed))
    return torch.randint(0, num_labels, (n,), generator=gen, device=device, dtype=torch.int64).to(torch.int32)
