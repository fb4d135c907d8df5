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
   whole graph.  Pairs that would make a self-loop, a repeated edge or (for
   external stubs) an edge inside one community are rejected and rewired: the
   rejected stubs are paired again and each new pair swaps ends with a random
   existing edge of the same kind, which keeps every degree.  Stubs still
   rejected after 40 rounds are dropped (well under 0.1 % of them at the
   benchmark sizes; the generator's stats report how many).
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

    # 4. wiring: internal stubs inside each community, external stubs across the graph,
    # then rejected stubs rewired into existing edges (see _rewire)
    stubs = torch.repeat_interleave(torch.arange(n, device=device), kin)
    key = labels[stubs] * (1 << 31) + _randint(gen, 1 << 31, stubs.numel(), device)
    stubs = stubs[torch.argsort(key)]
    del key
    ia, ib, left_in = _pair_stubs(stubs, labels, n, internal=True)
    del stubs
    stubs = torch.repeat_interleave(torch.arange(n, device=device), kout)
    stubs = stubs[torch.randperm(stubs.numel(), generator=gen, device=device)]
    ea, eb, left_ex = _pair_stubs(stubs, labels, n, internal=False)
    del stubs
    ia, ib, left_in, ea, eb, left_ex = _rewire(ia, ib, left_in, ea, eb, left_ex, labels, n, K, gen)
    dropped = int(left_in.numel() + left_ex.numel())
    lo = torch.cat([torch.minimum(ia, ib), torch.minimum(ea, eb)])
    hi = torch.cat([torch.maximum(ia, ib), torch.maximum(ea, eb)])
    del ia, ib, ea, eb
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
        "stubs_drawn": int(k.sum()),
        "stubs_dropped": dropped,
    }
    return graph


def _ukey(a: torch.Tensor, b: torch.Tensor, n: int) -> torch.Tensor:
    return torch.minimum(a, b) * n + torch.maximum(a, b)


def _first_of_equal(keys: torch.Tensor) -> torch.Tensor:
    """Mask of the first occurrence of every value in keys (by position)."""
    if keys.numel() == 0:
        return torch.zeros(0, dtype=torch.bool, device=keys.device)
    sk, idx = torch.sort(keys, stable=True)
    head = torch.ones_like(sk, dtype=torch.bool)
    head[1:] = sk[1:] != sk[:-1]
    keep = torch.zeros_like(head)
    keep[idx[head]] = True
    return keep


def _pair_stubs(stubs: torch.Tensor, labels: torch.Tensor, n: int, internal: bool):
    """Pair consecutive stubs; returns the valid simple edges (a, b) and the stubs of the
    rejected pairs: self-loops, repeats of an edge already formed, and pairs whose ends
    are in different communities (internal) or in the same one (external)."""
    odd = stubs[-1:] if stubs.numel() % 2 else stubs[:0]
    a, b = stubs[0:stubs.numel() - odd.numel():2], stubs[1:stubs.numel() - odd.numel():2]
    same = labels[a] == labels[b]
    ok = (same if internal else ~same) & (a != b)
    ok &= _first_of_equal(torch.where(ok, _ukey(a, b, n), -1 - torch.arange(a.numel(), device=a.device)))
    left = torch.cat([a[~ok], b[~ok], odd])
    return a[ok], b[ok], left


def _rewire(ia, ib, left_in, ea, eb, left_ex, labels, n: int, K: int, gen, rounds: int = 40):
    """Give rejected stubs an edge, as the LFR program does, without changing any degree:
    the rejected stubs are paired again at random (inside their community for internal
    stubs), and each such pair (a, b) replaces a random existing edge (x, y) of the same
    kind (internal edges of the same community, or external edges) by (a, x) and (b, y).
    A replacement is taken only if both new edges are simple, new and of the right kind;
    replacements that pick the same existing edge or form the same new edge are
    resolved in favour of the first.  Stubs still rejected after the last round are
    dropped."""
    device = labels.device
    for _ in range(rounds):
        if left_in.numel() < 2 and left_ex.numel() < 2:
            break
        exist = torch.sort(torch.cat([_ukey(ia, ib, n), _ukey(ea, eb, n)])).values
        moved = 0
        # internal: pair leftovers inside their community, swap with an internal edge of it
        if left_in.numel() >= 2 and ia.numel() > 0:
            key = labels[left_in] * (1 << 31) + _randint(gen, 1 << 31, left_in.numel(), device)
            s = left_in[torch.argsort(key)]
            odd = s[-1:] if s.numel() % 2 else s[:0]
            a, b = s[0:s.numel() - odd.numel():2], s[1:s.numel() - odd.numel():2]
            pair_ok = labels[a] == labels[b]
            rest = torch.cat([a[~pair_ok], b[~pair_ok], odd])
            a, b = a[pair_ok], b[pair_ok]
            c = labels[a]
            el = labels[ia]
            eo = torch.argsort(el, stable=True)
            cnt = torch.bincount(el, minlength=K)
            off = torch.cumsum(cnt, 0) - cnt
            has = cnt[c] > 0
            rest = torch.cat([rest, a[~has], b[~has]])
            a, b, c = a[has], b[has], c[has]
            r = (torch.rand(c.numel(), generator=gen, device=device, dtype=torch.float64) * cnt[c].to(torch.float64)).long()
            pick = eo[off[c] + torch.minimum(r, cnt[c] - 1)]
            ia, ib, a, b, done = _swap(ia, ib, pick, a, b, labels, n, exist, internal=True, gen=gen)
            left_in = torch.cat([rest, a[~done], b[~done]])
            moved += int(done.sum())
        # external: pair leftovers anywhere, swap with a random external edge
        if left_ex.numel() >= 2 and ea.numel() > 0:
            s = left_ex[torch.randperm(left_ex.numel(), generator=gen, device=device)]
            odd = s[-1:] if s.numel() % 2 else s[:0]
            a, b = s[0:s.numel() - odd.numel():2], s[1:s.numel() - odd.numel():2]
            pick = _randint(gen, ea.numel(), a.numel(), device)
            ea, eb, a, b, done = _swap(ea, eb, pick, a, b, labels, n, exist, internal=False, gen=gen)
            left_ex = torch.cat([odd, a[~done], b[~done]])
            moved += int(done.sum())
        if moved == 0:
            break
    return ia, ib, left_in, ea, eb, left_ex


def _swap(ea, eb, pick, a, b, labels, n: int, exist, internal: bool, gen):
    """Replace edge pick[p] = (x, y) by (a[p], x) and (b[p], y) where allowed; returns the
    new edge lists, the proposals (a, b) and the mask of those carried out."""
    device = a.device
    x, y = ea[pick], eb[pick]
    flip = torch.rand(a.numel(), generator=gen, device=device) < 0.5
    x, y = torch.where(flip, y, x), torch.where(flip, x, y)
    k1, k2 = _ukey(a, x, n), _ukey(b, y, n)
    ok = (a != x) & (b != y) & (k1 != k2)
    if internal:
        ok &= (labels[a] == labels[x]) & (labels[b] == labels[y])
    else:
        ok &= (labels[a] != labels[x]) & (labels[b] != labels[y])
    for kk in (k1, k2):
        pos = torch.searchsorted(exist, kk).clamp_(max=max(exist.numel() - 1, 0))
        ok &= exist[pos] != kk
    idx = torch.arange(a.numel(), device=device)
    # one replacement per existing edge
    ok &= _first_of_equal(torch.where(ok, pick, -1 - idx))
    # new edges distinct among themselves: a proposal is dropped if either edge repeats
    both = torch.cat([torch.where(ok, k1, -1 - idx), torch.where(ok, k2, -1 - a.numel() - idx)])
    sk, order = torch.sort(both)
    dup = torch.zeros_like(sk, dtype=torch.bool)
    dup[1:] |= sk[1:] == sk[:-1]
    dup[:-1] |= sk[1:] == sk[:-1]
    bad = torch.zeros_like(both, dtype=torch.bool)
    bad[order] = dup
    ok &= ~(bad[: a.numel()] | bad[a.numel():])
    keep = torch.ones(ea.numel(), dtype=torch.bool, device=device)
    keep[pick[ok]] = False
    na = torch.cat([ea[keep], a[ok], b[ok]])
    nb = torch.cat([eb[keep], x[ok], y[ok]])
    return na, nb, a, b, ok


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
