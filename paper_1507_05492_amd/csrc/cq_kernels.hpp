// cq_kernels.hpp -- gfx950 kernels of the community-quality library.
//
// Scoring one partition (Section II-B of the paper) runs as:
//   node pass   -> per-label size |c| and degree sum D_c = 2|E_c^in| + |E_c^out|, and for
//                  every node its slot inside its community's segment (counting sort)
//   scan/order  -> segment starts; non-empty communities ordered by decreasing D_c
//   edge pass   -> for every CSR entry (u, v) the label of v is written into the segment
//                  of u's community (streamed col_idx, gathered labels)
//   group pass  -> one workgroup per community counts its segment in LDS: the count of
//                  its own label is 2|E_c^in|, the others are |E_{c,c'}| (Eq. 9)
//   final       -> Q (Eq. 8), Qds (Eq. 9), the six measures (Section II-B3)
// Comparing two partitions (Section II-A) reuses the node pass (weight 1), scan and
// group pass on the contingency table rows: the segment of ground-truth community c_i
// holds the detected labels of its members, so the LDS counts are |c_i ∩ c'_j|.
#pragma once
#include "cq_device.hpp"

namespace cq {

// ---------------------------------------------------------------------------
// utility
__global__ void k_fill_u32(u32* __restrict__ p, size_t count, u32 v) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (size_t)gridDim.x * blockDim.x) p[i] = v;
}

// floor(log2(x)) + 1 for x > 0, 0 for x = 0
__device__ __forceinline__ int size_bucket_u32(u32 x) { return x ? 32 - __clz(x) : 0; }

// ---------------------------------------------------------------------------
// Graph checks (load time).  Structural: offsets monotone and within [0, nnz],
// indices within [0, n).  Full: no self-loops, rows strictly increasing (sorted, no
// repeated entry), and every (u, v) has its mirror (v, u).
// It also counts the degrees in power-of-two bins: bins[b] gets the rows with
// floor(log2(deg)) = b - 1 (bins[0]: the rows without entries).
constexpr int DEG_BINS = 32;
__global__ void k_check_csr(int n, long long nnz, const int32_t* __restrict__ rp, const int32_t* __restrict__ col,
                            u32* __restrict__ flags, u32* __restrict__ maxdeg, u32* __restrict__ bins) {
  __shared__ u32 s_bins[DEG_BINS];
  if (threadIdx.x < DEG_BINS) s_bins[threadIdx.x] = 0;
  __syncthreads();
  u32 bad = 0, md = 0;
  size_t stride = (size_t)gridDim.x * blockDim.x;
  for (size_t u = (size_t)blockIdx.x * blockDim.x + threadIdx.x; u < (size_t)n; u += stride) {
    long long a = rp[u], b = rp[u + 1];
    if (a < 0 || b < a || b > nnz) {
      bad = 1;
    } else {
      md = max(md, (u32)(b - a));
      atomicAdd(&s_bins[size_bucket_u32((u32)(b - a))], 1u);
    }
  }
  __syncthreads();
  if (threadIdx.x < DEG_BINS && s_bins[threadIdx.x]) atomicAdd(&bins[threadIdx.x], s_bins[threadIdx.x]);
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < (size_t)nnz; e += stride) {
    int v = col[e];
    if (v < 0 || v >= n) bad = 1;
  }
  md = wave_max_u32(md);
  if ((threadIdx.x & 63) == 0 && md) atomicMax(maxdeg, md);
  if (bad) atomicOr(flags, F_GRAPH);
}

__global__ void k_check_symmetric(int n, const int32_t* __restrict__ rp, const int32_t* __restrict__ col,
                                  const float* __restrict__ w, u32* __restrict__ flags) {
  // one wave per row; lanes stride over the row's entries
  int lane = threadIdx.x & 63;
  size_t wave = ((size_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  size_t nwaves = ((size_t)gridDim.x * blockDim.x) >> 6;
  u32 bad = 0;
  for (size_t u = wave; u < (size_t)n; u += nwaves) {
    int a = rp[u], b = rp[u + 1];
    for (int e = a + lane; e < b; e += 64) {
      int v = col[e];
      if (v == (int)u) bad = 1;
      if (e > a && col[e - 1] >= v) bad = 1;
      int lo = rp[v], hi = rp[v + 1];
      while (lo < hi) {  // lower_bound of u in the (sorted) row of v
        int mid = (lo + hi) >> 1;
        if (col[mid] < (int)u) lo = mid + 1; else hi = mid;
      }
      if (lo >= rp[v + 1] || col[lo] != (int)u) bad = 1;
      else if (w && __float_as_uint(w[lo]) != __float_as_uint(w[e])) bad = 1;  // the two entries of an edge
    }
  }
  if (bad) atomicOr(flags, F_GRAPH);
}

// Edge weights: finite and in [WEIGHT_MIN, WEIGHT_MAX]; per-block exact sums of
// w * 2^55 (two words per block) for the total weight.
__global__ __launch_bounds__(256) void k_check_weights(long long nnz, const float* __restrict__ w, u32* __restrict__ flags,
                                                       u64* __restrict__ parts) {
  __shared__ u64 s_lo[4], s_hi[4];
  u32 bad = 0;
  u128 sum = 0;
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < (size_t)nnz; e += stride) {
    const float x = w[e];
    if (!(x >= WEIGHT_MIN && x <= WEIGHT_MAX)) bad = 1;  // also catches NaN
    else sum += fixw_f32(x);
  }
  sum = wave_sum_u128(sum);
  const int wv = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    s_lo[wv] = (u64)sum;
    s_hi[wv] = (u64)(sum >> 64);
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    u128 t = 0;
    for (int i = 0; i < (int)(blockDim.x >> 6); ++i) t += ((u128)s_hi[i] << 64) | s_lo[i];
    parts[2 * blockIdx.x] = (u64)t;
    parts[2 * blockIdx.x + 1] = (u64)(t >> 64);
  }
  if (bad) atomicOr(flags, F_GRAPH);
}

// ---------------------------------------------------------------------------
// Exclusive scan of a u32 array of any length (three launches): tiles of
// SCAN_TILE items are scanned in place, the tile totals are scanned by one block,
// and the tile offsets are added back.  out[n] receives the total.
constexpr int SCAN_THREADS = 1024;
constexpr int SCAN_ITEMS = 4;
constexpr int SCAN_TILE = SCAN_THREADS * SCAN_ITEMS;

__device__ u32 block_excl_scan_1024(u32 x, u32* s_w, u32* total) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  u32 incl = wave_incl_scan(x);
  if (lane == 63) s_w[wv] = incl;
  __syncthreads();
  u32 before = 0, tot = 0;
  for (int i = 0; i < SCAN_THREADS / 64; ++i) {
    u32 t = s_w[i];
    if (i < wv) before += t;
    tot += t;
  }
  __syncthreads();
  *total = tot;
  return before + incl - x;
}

__global__ __launch_bounds__(SCAN_THREADS) void k_scan_tiles(long long n, const u32* __restrict__ in, u32* __restrict__ out,
                                                             u32* __restrict__ tile_sums) {
  __shared__ u32 s_w[SCAN_THREADS / 64];
  const long long base = (long long)blockIdx.x * SCAN_TILE + (long long)threadIdx.x * SCAN_ITEMS;
  u32 v[SCAN_ITEMS], sum = 0;
#pragma unroll
  for (int k = 0; k < SCAN_ITEMS; ++k) {
    v[k] = (base + k < n) ? in[base + k] : 0u;
    sum += v[k];
  }
  u32 total;
  u32 run = block_excl_scan_1024(sum, s_w, &total);
#pragma unroll
  for (int k = 0; k < SCAN_ITEMS; ++k) {
    if (base + k < n) out[base + k] = run;
    run += v[k];
  }
  if (threadIdx.x == 0) tile_sums[blockIdx.x] = total;
}

__global__ __launch_bounds__(SCAN_THREADS) void k_scan_tops(int T, u32* __restrict__ tile_sums, long long n, u32* __restrict__ out) {
  __shared__ u32 s_w[SCAN_THREADS / 64];
  __shared__ u32 s_carry;
  if (threadIdx.x == 0) s_carry = 0;
  __syncthreads();
  for (int b = 0; b < T; b += SCAN_THREADS) {
    int i = b + threadIdx.x;
    u32 x = i < T ? tile_sums[i] : 0u;
    u32 total;
    u32 ex = block_excl_scan_1024(x, s_w, &total);
    u32 carry = s_carry;
    if (i < T) tile_sums[i] = carry + ex;
    __syncthreads();
    if (threadIdx.x == 0) s_carry = carry + total;
    __syncthreads();
  }
  if (threadIdx.x == 0) out[n] = s_carry;
}

__global__ __launch_bounds__(SCAN_THREADS) void k_scan_add(long long n, u32* __restrict__ out, const u32* __restrict__ tile_sums) {
  const long long base = (long long)blockIdx.x * SCAN_TILE + (long long)threadIdx.x * SCAN_ITEMS;
  const u32 off = tile_sums[blockIdx.x];
#pragma unroll
  for (int k = 0; k < SCAN_ITEMS; ++k)
    if (base + k < n) out[base + k] += off;
}

// ---------------------------------------------------------------------------
// Locality order for a graph (load time, graph only).  A few sweeps of label
// propagation group nodes into clusters; nodes are then renumbered cluster by
// cluster, so that most neighbours of a row have nearby ids.  The order only moves
// data: every count the library reports is the same in any node order.
constexpr u32 HMUL = 0x9E3779B1u;  // odd, so x -> x*HMUL is a bijection on 32-bit words
constexpr u32 HINV = 0x0E8B2F51u;  // HMUL * HINV == 1 (mod 2^32)
constexpr int LP_CAP = 256;         // neighbours looked at per row

__global__ void k_iota(int n, int32_t* __restrict__ a) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < (size_t)n; i += (size_t)gridDim.x * blockDim.x) a[i] = (int32_t)i;
}

// One sweep: every node takes the label that occurs most often among (up to LP_CAP of)
// its neighbours; ties go to the label with the smallest hash.  One wave per row.
__global__ __launch_bounds__(256) void k_lp(int n, const int32_t* __restrict__ rp, const int32_t* __restrict__ col,
                                            const int32_t* __restrict__ lin, int32_t* __restrict__ lout, int sweep) {
  const int lane = threadIdx.x & 63;
  const size_t wave = ((size_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const size_t nwaves = ((size_t)gridDim.x * blockDim.x) >> 6;
  for (size_t u = wave; u < (size_t)n; u += nwaves) {
    const int a = rp[u];
    const int deg = min(rp[u + 1] - a, LP_CAP);
    // ties between labels: a fixed order of labels (sweep < 0), or one salted per node
    // and sweep, so that no label wins every tie
    const u32 salt = sweep < 0 ? 0u : (((u32)u * 0x85EBCA6Bu) ^ ((u32)sweep * 0xC2B2AE35u));
    if (deg == 0) {
      if (lane == 0) lout[u] = lin[u];
      continue;
    }
    int x[LP_CAP / 64];
    u32 cnt[LP_CAP / 64];
#pragma unroll
    for (int q = 0; q < LP_CAP / 64; ++q) {
      const int k = lane + 64 * q;
      x[q] = k < deg ? lin[col[a + k]] : -1;
      cnt[q] = 0;
    }
    const int chunks = (deg + 63) >> 6;
    for (int q2 = 0; q2 < chunks; ++q2) {
      const int lim = min(64, deg - 64 * q2);
      int xv = x[0];
#pragma unroll
      for (int q = 1; q < LP_CAP / 64; ++q) if (q == q2) xv = x[q];
      for (int s2 = 0; s2 < lim; ++s2) {
        const int y = __shfl(xv, s2, 64);
#pragma unroll
        for (int q = 0; q < LP_CAP / 64; ++q) cnt[q] += (x[q] == y) ? 1u : 0u;
      }
    }
    u64 best = 0;
#pragma unroll
    for (int q = 0; q < LP_CAP / 64; ++q) {
      if (x[q] >= 0) {
        const u64 key = ((u64)cnt[q] << 32) | (u64)(~(((u32)x[q] ^ salt) * HMUL));
        best = key > best ? key : best;
      }
    }
    best = wave_max_u64(best);
    if (lane == 0) lout[u] = (int32_t)(((~(u32)best) * HINV) ^ salt);
  }
}

__global__ void k_count_labels(int n, const int32_t* __restrict__ lab, u32* __restrict__ cnt) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < (size_t)n; i += (size_t)gridDim.x * blockDim.x)
    atomicAdd(&cnt[lab[i]], 1u);
}

// out[0] += number of non-empty clusters, out[1] = largest cluster (one atomic per wave)
__global__ void k_cluster_stats(int n, const u32* __restrict__ cnt, u32* __restrict__ out) {
  for (size_t b = (size_t)blockIdx.x * blockDim.x; b < (size_t)n; b += (size_t)gridDim.x * blockDim.x) {  // uniform
    const size_t i = b + threadIdx.x;
    const u32 c = i < (size_t)n ? cnt[i] : 0u;
    const u64 nz = __ballot(c > 0);
    const u32 mx = wave_max_u32(c);
    if ((threadIdx.x & 63) == 0 && nz) {
      atomicAdd(&out[0], (u32)__popcll(nz));
      atomicMax(&out[1], mx);
    }
  }
}

// new id of node u = start[cluster] + arrival order inside the cluster
__global__ void k_place(int n, const int32_t* __restrict__ lab, const u32* __restrict__ start, u32* __restrict__ cursor,
                        int32_t* __restrict__ newid, int32_t* __restrict__ old) {
  for (size_t u = (size_t)blockIdx.x * blockDim.x + threadIdx.x; u < (size_t)n; u += (size_t)gridDim.x * blockDim.x) {
    const int c = lab[u];
    const u32 p = start[c] + atomicAdd(&cursor[c], 1u);
    newid[u] = (int32_t)p;
    old[p] = (int32_t)u;
  }
}

__global__ void k_new_degree(int n, const int32_t* __restrict__ rp, const int32_t* __restrict__ old, u32* __restrict__ deg) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < (size_t)n; i += (size_t)gridDim.x * blockDim.x) {
    const int u = old[i];
    deg[i] = (u32)(rp[u + 1] - rp[u]);
  }
}

// row i of the renumbered graph = row old[i] of the input, with neighbour ids renumbered
__global__ __launch_bounds__(256) void k_relabel_rows(int n, const int32_t* __restrict__ rp, const int32_t* __restrict__ col,
                                                      const int32_t* __restrict__ old, const int32_t* __restrict__ newid,
                                                      const int32_t* __restrict__ rp2, int32_t* __restrict__ col2,
                                                      const float* __restrict__ w, float* __restrict__ w2) {
  const int lane = threadIdx.x & 63;
  const size_t wave = ((size_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const size_t nwaves = ((size_t)gridDim.x * blockDim.x) >> 6;
  for (size_t i = wave; i < (size_t)n; i += nwaves) {
    const int u = old[i];
    const int a = rp[u], deg = rp[u + 1] - a, b = rp2[i];
    for (int k = lane; k < deg; k += 64) {
      col2[b + k] = newid[col[a + k]];
      if (w) w2[b + k] = w[a + k];
    }
  }
}

// Column blocks of the renumbered graph.  The id range is cut into COL_BLOCKS spans of
// `span` ids; block y holds, row by row, the entries whose neighbour lies in span y, as
// its own CSR whose row pointers RPB[y*(n+1) + u] index one array colb shared by all
// blocks (block y's entries follow block y-1's); rowb holds the row of every entry.
// One wave per row.
constexpr int COL_BLOCKS = 8;

__global__ __launch_bounds__(256) void k_blk_count(int n, const int32_t* __restrict__ rp, const int32_t* __restrict__ col,
                                                   int span, u32* __restrict__ cnt) {
  const int lane = threadIdx.x & 63;
  const size_t wave = ((size_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const size_t nwaves = ((size_t)gridDim.x * blockDim.x) >> 6;
  for (size_t u = wave; u < (size_t)n; u += nwaves) {
    const int a = rp[u], deg = rp[u + 1] - a;
    u32 mine = 0;  // lane y < COL_BLOCKS counts block y
    for (int k0 = 0; k0 < deg; k0 += 64) {
      const int y = k0 + lane < deg ? col[a + k0 + lane] / span : -1;
#pragma unroll
      for (int b = 0; b < COL_BLOCKS; ++b) {
        const u32 c = (u32)__popcll(__ballot(y == b));
        if (lane == b) mine += c;
      }
    }
    if (lane < COL_BLOCKS) cnt[(size_t)lane * ((size_t)n + 1) + u] = mine;
    if (u == 0 && lane < COL_BLOCKS) cnt[(size_t)lane * ((size_t)n + 1) + n] = 0;
  }
}

__global__ __launch_bounds__(256) void k_blk_place(int n, const int32_t* __restrict__ rp, const int32_t* __restrict__ col,
                                                   int span, const u32* __restrict__ RPB, int32_t* __restrict__ colb,
                                                   int32_t* __restrict__ rowb, const float* __restrict__ w,
                                                   float* __restrict__ wb) {
  const int lane = threadIdx.x & 63;
  const u64 below = lane ? (~0ull >> (64 - lane)) : 0ull;
  const size_t wave = ((size_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const size_t nwaves = ((size_t)gridDim.x * blockDim.x) >> 6;
  for (size_t u = wave; u < (size_t)n; u += nwaves) {
    const int a = rp[u], deg = rp[u + 1] - a;
    u32 fill_b = lane < COL_BLOCKS ? RPB[(size_t)lane * ((size_t)n + 1) + u] : 0u;  // lane y: next slot of block y
    for (int k0 = 0; k0 < deg; k0 += 64) {
      const bool in = k0 + lane < deg;
      const int v = in ? col[a + k0 + lane] : 0;
      const int y = in ? v / span : -1;
      u32 slot = 0;
#pragma unroll
      for (int b = 0; b < COL_BLOCKS; ++b) {
        const u64 m = __ballot(y == b);
        const u32 base = __shfl(fill_b, b, 64);
        if (y == b) slot = base + (u32)__popcll(m & below);
        if (lane == b) fill_b += (u32)__popcll(m);
      }
      if (in) {
        colb[slot] = v;
        rowb[slot] = (int32_t)u;
        if (w) wb[slot] = w[a + k0 + lane];
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Node pass, LDS-private histograms (num_labels small enough for LDS).
// Workgroup w owns nodes [w*chunk, (w+1)*chunk).  It counts, per label, the nodes
// (HN) and the weights (HD: degree when WEIGHTED, else 1) of its nodes, and gives
// each node the running weight offset of its label inside the workgroup (loc).
// Rows w of HN/HD are later prefix-summed over w, which turns loc into a position
// inside the label's segment.
template <class LT>
struct LabelT {
  static constexpr LT SENTINEL = (LT)~(LT)0;  // "no label" marker in staged label arrays
};

// Label permutation plan (load time).  Scoring calls receive labels in the caller's
// node order, the kernels want them in the stored order.  A random gather costs a
// whole cache line per label, so the move is done in two streaming passes instead:
// node u (caller order) first writes its label to tmp[pos1[u]], where tmp is grouped
// into buckets of 2^PERM_SHIFT stored ids (bucket b = newid >> PERM_SHIFT); then one
// workgroup per bucket copies every slot j of bucket b to labx[b * 2^PERM_SHIFT + tgt[j]]
// through LDS (the bucket's labels fit there; tgt holds the 16-bit offset of the stored
// id in its bucket) and writes the bucket's labels out in order.  The order inside a
// bucket is whatever the atomics gave.
constexpr int PERM_SHIFT = 15;  // 32768 stored ids per bucket: 64 KB of 16-bit labels

// Each workgroup counts its nodes per bucket in LDS, reserves a range of every bucket
// with one global atomic, and places its nodes inside those ranges.
constexpr int PERM_NODES = 8192;  // nodes per workgroup of the plan kernels
constexpr int PERM_MAX_BUCKETS = 16384;  // n up to 2^29

__global__ __launch_bounds__(256) void k_perm_count(int n, const int32_t* __restrict__ newid, int nb, u32* __restrict__ bcnt) {
  __shared__ u32 h[PERM_MAX_BUCKETS];
  for (int i = threadIdx.x; i < nb; i += blockDim.x) h[i] = 0;
  __syncthreads();
  const long long u0 = (long long)blockIdx.x * PERM_NODES, u1 = min((long long)n, u0 + PERM_NODES);
  for (long long u = u0 + threadIdx.x; u < u1; u += blockDim.x) atomicAdd(&h[(u32)newid[u] >> PERM_SHIFT], 1u);
  __syncthreads();
  for (int i = threadIdx.x; i < nb; i += blockDim.x)
    if (h[i]) atomicAdd(&bcnt[i], h[i]);
}

// With lrank/spos (column-blocked graphs): the workgroup's slots in bucket order are
// numbered 0 .. PERM_NODES-1 (its ranges of buckets 0, 1, ... one after the other);
// lrank[u] is node u's number and spos[u0 + r] the slot numbered r, so a pass that puts
// the chunk's labels in LDS by number writes them out to consecutive slots.
__global__ __launch_bounds__(256) void k_perm_plan(int n, const int32_t* __restrict__ newid, int nb,
                                                   const u32* __restrict__ bstart, u32* __restrict__ bcur,
                                                   u32* __restrict__ pos1, uint16_t* __restrict__ tgt,
                                                   uint16_t* __restrict__ lrank, u32* __restrict__ spos) {
  extern __shared__ u32 plan_sh[];
  u32* h = plan_sh;        // counts, then the next slot of each range
  u32* d = plan_sh + nb;   // first slot of range i minus the number of its first slot
  __shared__ u32 s_part[256];
  for (int i = threadIdx.x; i < nb; i += blockDim.x) h[i] = 0;
  __syncthreads();
  const long long u0 = (long long)blockIdx.x * PERM_NODES, u1 = min((long long)n, u0 + PERM_NODES);
  for (long long u = u0 + threadIdx.x; u < u1; u += blockDim.x) atomicAdd(&h[(u32)newid[u] >> PERM_SHIFT], 1u);
  __syncthreads();
  // exclusive scan of the counts: thread t sums buckets [t*per, (t+1)*per)
  const int per = (nb + (int)blockDim.x - 1) / (int)blockDim.x;
  const int i0 = min(nb, (int)threadIdx.x * per), i1 = min(nb, i0 + per);
  u32 part = 0;
  for (int i = i0; i < i1; ++i) part += h[i];
  s_part[threadIdx.x] = part;
  __syncthreads();
  if (threadIdx.x == 0) {
    u32 run = 0;
    for (int t = 0; t < (int)blockDim.x; ++t) {
      const u32 x = s_part[t];
      s_part[t] = run;
      run += x;
    }
  }
  __syncthreads();
  {
    u32 first = s_part[threadIdx.x];
    for (int i = i0; i < i1; ++i) {
      const u32 c = h[i];
      const u32 base = c ? bstart[i] + atomicAdd(&bcur[i], c) : 0u;  // this workgroup's range in bucket i
      d[i] = base - first;
      h[i] = base;
      first += c;
    }
  }
  __syncthreads();
  for (long long u = u0 + threadIdx.x; u < u1; u += blockDim.x) {
    const u32 v = (u32)newid[u];
    const u32 b = v >> PERM_SHIFT;
    const u32 p = atomicAdd(&h[b], 1u);
    pos1[u] = p;
    tgt[p] = (uint16_t)(v & ((1u << PERM_SHIFT) - 1u));
    if (lrank) {
      const u32 r = p - d[b];  // < PERM_NODES
      lrank[u] = (uint16_t)r;
      spos[u0 + r] = p;
    }
  }
}

__global__ void k_degree(int n, const int32_t* __restrict__ rp, u32* __restrict__ deg) {
  for (size_t u = (size_t)blockIdx.x * blockDim.x + threadIdx.x; u < (size_t)n; u += (size_t)gridDim.x * blockDim.x)
    deg[u] = (u32)(rp[u + 1] - rp[u]);
}

// Node pass in the caller's order for a renumbered graph (labels fit LDS): workgroup w
// counts nodes and degrees per label over nodes [w*chunk, (w+1)*chunk) into its rows of
// HN/HD, and writes each label (or the sentinel) to tmp[pos1[u]].
template <class LT>
__global__ __launch_bounds__(1024) void k_node_perm(int n, const int32_t* __restrict__ labels, const u32* __restrict__ deg,
                                                    const u32* __restrict__ pos1, int L, int chunk, u32* __restrict__ HN,
                                                    u32* __restrict__ HD, LT* __restrict__ tmp, Ctl* __restrict__ ctl) {
  extern __shared__ u32 sh[];
  u32* hn = sh;
  u32* hd = sh + L;
  __shared__ u32 s_bad;
  for (int i = threadIdx.x; i < 2 * L; i += blockDim.x) sh[i] = 0;
  if (threadIdx.x == 0) s_bad = 0;
  __syncthreads();
  const long long u0 = (long long)blockIdx.x * chunk, u1 = min((long long)n, u0 + chunk);
  constexpr int U = 8;  // nodes per thread in flight
  u32 bad = 0;
  for (long long ub = u0 + threadIdx.x; ub < u1; ub += (long long)U * blockDim.x) {
    int c[U];
    u32 d[U], p[U];
#pragma unroll
    for (int k = 0; k < U; ++k) {
      const long long u = min(ub + (long long)k * blockDim.x, u1 - 1);  // in bounds; masked below
      c[k] = labels[u];
      d[k] = deg[u];
      p[k] = pos1[u];
    }
#pragma unroll
    for (int k = 0; k < U; ++k) {
      if (ub + (long long)k * blockDim.x >= u1) break;
      if ((u32)c[k] < (u32)L) {
        atomicAdd(&hn[c[k]], 1u);
        atomicAdd(&hd[c[k]], d[k]);
        tmp[p[k]] = (LT)c[k];
      } else {
        bad = 1;
        tmp[p[k]] = LabelT<LT>::SENTINEL;
      }
    }
  }
  if (bad) s_bad = 1;
  __syncthreads();
  const size_t row = (size_t)blockIdx.x * (size_t)L;
  for (int c = threadIdx.x; c < L; c += blockDim.x) {
    HN[row + c] = hn[c];
    HD[row + c] = hd[c];
  }
  if (threadIdx.x == 0 && s_bad) atomicOr(&ctl->flags, F_LABEL);
}

// Node pass of a column-blocked graph, in two kernels.  k_node_scatter moves the labels
// from the caller's order into the plan's buckets (tmp[pos1[u]]), one workgroup per
// PERM_NODES nodes, which own one range of every bucket: the labels go to LDS by their
// number in the plan (lrank) and leave in slot order (spos), so neighbouring lanes write
// neighbouring slots.  Its first threads also clear N and D.  k_perm_apply_count then
// moves each bucket to the stored order and counts nodes and degrees per label there,
// where the labels of a renumbered graph come in long runs.
template <class LT>
__global__ __launch_bounds__(1024) void k_node_scatter(int n, const int32_t* __restrict__ labels,
                                                       const uint16_t* __restrict__ lrank, const u32* __restrict__ spos,
                                                       int L, LT* __restrict__ tmp, u32* __restrict__ N, u32* __restrict__ D,
                                                       Ctl* __restrict__ ctl) {
  __shared__ LT s_lab[PERM_NODES];
  for (size_t c = (size_t)blockIdx.x * blockDim.x + threadIdx.x; c < (size_t)L; c += (size_t)gridDim.x * blockDim.x) {
    N[c] = 0;
    D[c] = 0;
  }
  constexpr int U = PERM_NODES / 1024;
  const long long u0 = (long long)blockIdx.x * PERM_NODES;
  const u32 cnt = (u32)min((long long)PERM_NODES, (long long)n - u0);
  int c[U];
  u32 r[U];
#pragma unroll
  for (int k = 0; k < U; ++k) {
    const long long u = min(u0 + k * 1024 + threadIdx.x, (long long)n - 1);  // in bounds; masked below
    c[k] = labels[u];
    r[k] = lrank[u];
  }
  u32 bad = 0;
#pragma unroll
  for (int k = 0; k < U; ++k) {
    if ((u32)(k * 1024) + threadIdx.x < cnt) {
      const bool ok = (u32)c[k] < (u32)L;
      bad |= ok ? 0u : 1u;
      s_lab[r[k]] = ok ? (LT)c[k] : LabelT<LT>::SENTINEL;
    }
  }
  if (bad) atomicOr(&ctl->flags, F_LABEL);
  __syncthreads();
  // numbers 0 .. cnt-1 are the chunk's slots in increasing order within each range
  for (u32 i = threadIdx.x; i < cnt; i += blockDim.x) tmp[spos[u0 + i]] = s_lab[i];
}

// Labels up to which k_perm_apply_count counts in LDS: 64 KB of 16-bit labels and two
// 32-bit counters per label, with its few static words, stay within a CU's 160 KB.
constexpr int APPLY_COUNT_MAX_L = 12224;
// A bucket with at most this many distinct labels adds its counts to N and D with
// global atomics; a denser one writes a histogram row instead (see k_colscan_rows).
constexpr u32 FLUSH_MAX = 256;

// Bucket b (one workgroup): labx[id] for its stored ids, as k_perm_apply, and per label
// the number of its nodes and the sum of their degrees (rp: stored-order row_ptr).
// Each thread takes 8 consecutive ids; a wave whose 512 ids carry one label adds them
// with one LDS atomic per counter.  Sentinels (out-of-range labels) are not counted.
__global__ __launch_bounds__(1024) void k_perm_apply_count(const u32* __restrict__ bstart, const uint16_t* __restrict__ tgt,
                                                           const uint16_t* __restrict__ tmp, uint16_t* __restrict__ labx,
                                                           const int32_t* __restrict__ rp, int L, u32* __restrict__ N,
                                                           u32* __restrict__ D, u32* __restrict__ HN, u32* __restrict__ HD,
                                                           u32* __restrict__ rows, Ctl* __restrict__ ctl) {
  extern __shared__ uint4 sl4[];
  uint16_t* sl = reinterpret_cast<uint16_t*>(sl4);
  u32* hn = reinterpret_cast<u32*>(sl4 + (1u << PERM_SHIFT) / 8u);
  u32* hd = hn + L;
  __shared__ u32 s_nz;
  __shared__ u32 s_chg;
  const int tid = threadIdx.x;
  const u32 b = blockIdx.x, id0 = b << PERM_SHIFT;
  const u32 j0 = bstart[b], j1 = bstart[b + 1];
  for (int i = tid; i < 2 * L; i += blockDim.x) hn[i] = 0;
  if (tid == 0) {
    s_nz = 0;
    s_chg = 0;
  }
  u32 chg = 0;  // label changes between consecutive stored ids of this bucket
  constexpr int U = 8;
  for (u32 jb = j0 + tid; jb < j1; jb += U * blockDim.x) {
    u32 t[U];
    uint16_t x[U];
#pragma unroll
    for (int k = 0; k < U; ++k) {
      const u32 j = min(jb + (u32)k * blockDim.x, j1 - 1u);  // in bounds; masked below
      t[k] = tgt[j];
      x[k] = tmp[j];
    }
#pragma unroll
    for (int k = 0; k < U; ++k)
      if (jb + (u32)k * blockDim.x < j1) sl[t[k]] = x[k];
  }
  __syncthreads();
  // the bucket's ids [id0, id0 + cnt) are all present exactly once: write them in order
  const u32 cnt = j1 - j0, nv = cnt / 8u;
  uint4* dst = reinterpret_cast<uint4*>(labx + id0);  // id0 is a multiple of 2^PERM_SHIFT: 16-byte aligned
  for (u32 v0 = 0; v0 < nv; v0 += blockDim.x) {  // the same trip count for every lane of a wave
    const u32 i = v0 + (u32)tid;
    const bool act = i < nv;
    uint4 q = make_uint4(0u, 0u, 0u, 0u);
    int r[9];
    if (act) {
      q = sl4[i];
      dst[i] = q;
      const int32_t* rr = rp + id0 + 8u * i;  // ids id0+8i .. id0+8i+7 and the next row start (<= n)
#pragma unroll
      for (int k = 0; k < 9; ++k) r[k] = rr[k];
    } else {
#pragma unroll
      for (int k = 0; k < 9; ++k) r[k] = 0;
    }
    const u32 w4[4] = {q.x, q.y, q.z, q.w};
    const u32 l0 = q.x & 0xFFFFu;
    bool same = act;
#pragma unroll
    for (int k = 1; k < 8; ++k) same = same && ((w4[k >> 1] >> (16 * (k & 1))) & 0xFFFFu) == l0;
    if (act) {
      u32 prev = i ? (u32)sl[8u * i - 1u] : l0;
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        const u32 lk = (w4[k >> 1] >> (16 * (k & 1))) & 0xFFFFu;
        chg += lk != prev ? 1u : 0u;
        prev = lk;
      }
    }
    const u32 key = (same && l0 < (u32)L) ? l0 : 0xFFFFFFFFu;
    const u32 k0 = __shfl(key, 0, 64);
    if (__ballot(key == k0) == ~0ull && k0 != 0xFFFFFFFFu) {
      const u64 ds = wave_sum_u64((u64)(u32)(r[8] - r[0]));
      if ((tid & 63) == 0) {
        atomicAdd(&hn[k0], 512u);
        atomicAdd(&hd[k0], (u32)ds);
      }
    } else if (act) {
      if (key != 0xFFFFFFFFu) {
        atomicAdd(&hn[key], 8u);
        atomicAdd(&hd[key], (u32)(r[8] - r[0]));
      } else {
#pragma unroll
        for (int k = 0; k < 8; ++k) {
          const u32 lk = (w4[k >> 1] >> (16 * (k & 1))) & 0xFFFFu;
          if (lk < (u32)L) {
            atomicAdd(&hn[lk], 1u);
            atomicAdd(&hd[lk], (u32)(r[k + 1] - r[k]));
          }
        }
      }
    }
  }
  for (u32 i = nv * 8u + tid; i < cnt; i += blockDim.x) {
    const u32 lk = sl[i];
    chg += (i && lk != (u32)sl[i - 1u]) ? 1u : 0u;
    labx[id0 + i] = (uint16_t)lk;
    if (lk < (u32)L) {
      atomicAdd(&hn[lk], 1u);
      atomicAdd(&hd[lk], (u32)(rp[id0 + i + 1] - rp[id0 + i]));
    }
  }
  chg = (u32)wave_sum_u64(chg);
  if ((tid & 63) == 0 && chg) atomicAdd(&s_chg, chg);
  __syncthreads();
  u32 nz = 0;
  for (int c = tid; c < L; c += blockDim.x) nz += hn[c] ? 1u : 0u;
  nz = (u32)wave_sum_u64(nz);
  if ((tid & 63) == 0 && nz) atomicAdd(&s_nz, nz);
  __syncthreads();
  if (tid == 0 && s_chg) atomicAdd(&ctl->changes, s_chg);
  if (s_nz <= FLUSH_MAX) {
    for (int c = tid; c < L; c += blockDim.x) {
      if (hn[c]) {
        atomicAdd(&N[c], hn[c]);
        atomicAdd(&D[c], hd[c]);
      }
    }
  } else {
    const size_t row = (size_t)b * (size_t)L;
    for (int c = tid; c < L; c += blockDim.x) {
      HN[row + c] = hn[c];
      HD[row + c] = hd[c];
    }
    if (tid == 0) rows[atomicAdd(&ctl->dense_rows, 1u)] = b;
  }
}

// Caller-order pass without counting (labels beyond LDS, or a graph without column
// blocks): tmp[pos1[u]] = label of u, or the sentinel (flagged) when out of range.
template <class LT>
__global__ __launch_bounds__(256) void k_perm_scatter(int n, const int32_t* __restrict__ labels, const u32* __restrict__ pos1,
                                                      int L, LT* __restrict__ tmp, Ctl* __restrict__ ctl) {
  constexpr int U = 8;
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  u32 bad = 0;
  for (size_t ub = (size_t)blockIdx.x * blockDim.x + threadIdx.x; ub < (size_t)n; ub += U * stride) {
    int c[U];
    u32 p[U];
#pragma unroll
    for (int k = 0; k < U; ++k) {
      const size_t u = min(ub + k * stride, (size_t)n - 1);  // in bounds; masked below
      c[k] = labels[u];
      p[k] = pos1[u];
    }
#pragma unroll
    for (int k = 0; k < U; ++k) {
      if (ub + k * stride >= (size_t)n) break;
      const bool ok = (u32)c[k] < (u32)L;
      bad |= ok ? 0u : 1u;
      tmp[p[k]] = ok ? (LT)c[k] : LabelT<LT>::SENTINEL;
    }
  }
  if (bad) atomicOr(&ctl->flags, F_LABEL);
}

// The same move in two streaming passes, for graphs without column blocks: caller-order
// labels scattered straight to their buckets land on random cache lines (one partial line
// per 2-byte write over the whole label array).  Stored ids are cut into super-buckets of
// 2^SB_SHIFT (2 MB of 16-bit labels, one XCD's L2).
//   k_perm_split: a workgroup takes PS_NODES caller-order nodes, sorts them by super-bucket
//   in LDS and writes each super-bucket's run, one claim per run, into that super-bucket's
//   region of a 64-bit staging array: (super-bucket << 52) | (offset << 32) | label.
//   k_perm_place: the workgroups of a super-bucket, all on one XCD, write its labels to
//   their stored ids, random 2-byte writes inside one 2 MB range.
// sid[u] is the stored id of caller node u (a bijection onto [0, n)), so super-bucket b
// receives exactly min(2^SB_SHIFT, n - b * 2^SB_SHIFT) words.
constexpr int SB_SHIFT = 20;
constexpr u32 SB_MASK = (1u << SB_SHIFT) - 1u;
constexpr int SB_MAX = 1024;  // super-buckets (n <= 2^30): one per thread of k_perm_split's scan
constexpr int PS_NPT = 8;
constexpr int PS_NODES = 1024 * PS_NPT;
constexpr int PP_NPT = 16;
constexpr u32 PP_PARTS = (1u << SB_SHIFT) / (1024u * PP_NPT);  // k_perm_place workgroups per super-bucket

template <class LT>
__global__ __launch_bounds__(1024) void k_perm_split(int n, const int32_t* __restrict__ labels, const u32* __restrict__ sid,
                                                     int L, int nsb, u32* __restrict__ gcur,
                                                     unsigned long long* __restrict__ stage, Ctl* __restrict__ ctl) {
  __shared__ unsigned long long s_stage[PS_NODES];
  __shared__ u32 s_cnt[SB_MAX], s_off[SB_MAX], s_base[SB_MAX];
  __shared__ u32 s_w[SCAN_THREADS / 64];
  const int tid = threadIdx.x;
  const long long u0 = (long long)blockIdx.x * PS_NODES;
  s_cnt[tid] = 0;
  __syncthreads();
  int c[PS_NPT];
  u32 sv[PS_NPT];
#pragma unroll
  for (int k = 0; k < PS_NPT; ++k) {
    const long long u = min(u0 + tid + (long long)k * 1024, (long long)n - 1);  // in bounds; masked below
    c[k] = labels[u];
    sv[k] = sid[u];
  }
  unsigned long long wd[PS_NPT];
  u32 sb[PS_NPT], rank[PS_NPT];
  u32 bad = 0;
#pragma unroll
  for (int k = 0; k < PS_NPT; ++k) {
    sb[k] = 0xFFFFFFFFu;
    if (u0 + tid + (long long)k * 1024 < (long long)n) {
      const bool ok = (u32)c[k] < (u32)L;
      bad |= ok ? 0u : 1u;
      const u32 lab = ok ? (u32)(LT)c[k] : (u32)LabelT<LT>::SENTINEL;
      sb[k] = sv[k] >> SB_SHIFT;
      wd[k] = ((unsigned long long)sb[k] << 52) | ((unsigned long long)(sv[k] & SB_MASK) << 32) | lab;
    }
  }
#pragma unroll
  for (int k = 0; k < PS_NPT; ++k)
    if (sb[k] != 0xFFFFFFFFu) rank[k] = atomicAdd(&s_cnt[sb[k]], 1u);
  __syncthreads();
  const u32 cnt = s_cnt[tid];
  u32 total;
  s_off[tid] = block_excl_scan_1024(cnt, s_w, &total);
  s_base[tid] = (tid < nsb && cnt) ? atomicAdd(&gcur[tid], cnt) : 0u;  // one claim per run
  __syncthreads();
#pragma unroll
  for (int k = 0; k < PS_NPT; ++k)
    if (sb[k] != 0xFFFFFFFFu) s_stage[s_off[sb[k]] + rank[k]] = wd[k];
  __syncthreads();
  for (u32 p = tid; p < total; p += 1024) {
    const unsigned long long w = s_stage[p];
    const u32 b = (u32)(w >> 52);
    stage[((size_t)b << SB_SHIFT) + s_base[b] + (p - s_off[b])] = w;
  }
  if (bad) atomicOr(&ctl->flags, F_LABEL);
}

// Workgroup b runs on XCD b % 8 and takes part (b / 8) % PP_PARTS of super-bucket
// b % 8 + 8 * ((b / 8) / PP_PARTS).
template <class LT>
__global__ __launch_bounds__(1024) void k_perm_place(int n, int nsb, const unsigned long long* __restrict__ stage,
                                                     LT* __restrict__ labx) {
  const u32 x = blockIdx.x % 8u, i = blockIdx.x / 8u;
  const u32 b = x + 8u * (i / PP_PARTS), part = i % PP_PARTS;
  if (b >= (u32)nsb) return;
  const size_t s0 = (size_t)b << SB_SHIFT;
  const u32 size = (u32)min((size_t)1 << SB_SHIFT, (size_t)n - s0);
  const u32 e0 = part * 1024u * PP_NPT;
  if (e0 >= size) return;
  constexpr unsigned long long LMASK = sizeof(LT) == 2 ? 0xFFFFull : 0xFFFFFFFFull;
  unsigned long long w[PP_NPT];
#pragma unroll
  for (int k = 0; k < PP_NPT; ++k) w[k] = stage[s0 + min(e0 + threadIdx.x + (u32)k * 1024u, size - 1u)];  // masked below
#pragma unroll
  for (int k = 0; k < PP_NPT; ++k)
    if (e0 + threadIdx.x + (u32)k * 1024u < size) labx[s0 + (u32)((w[k] >> 32) & SB_MASK)] = (LT)(w[k] & LMASK);
}

template <class LT>
__global__ __launch_bounds__(1024) void k_perm_apply(int n, const u32* __restrict__ bstart, const uint16_t* __restrict__ tgt,
                                                     const LT* __restrict__ tmp, LT* __restrict__ labx) {
  extern __shared__ uint4 sl4[];
  LT* sl = reinterpret_cast<LT*>(sl4);
  const u32 b = blockIdx.x, id0 = b << PERM_SHIFT;
  const u32 j0 = bstart[b], j1 = bstart[b + 1];
  constexpr int U = 8;
  for (u32 jb = j0 + threadIdx.x; jb < j1; jb += U * blockDim.x) {
    u32 t[U];
    LT x[U];
#pragma unroll
    for (int k = 0; k < U; ++k) {
      const u32 j = min(jb + (u32)k * blockDim.x, j1 - 1u);  // in bounds; masked below
      t[k] = tgt[j];
      x[k] = tmp[j];
    }
#pragma unroll
    for (int k = 0; k < U; ++k)
      if (jb + (u32)k * blockDim.x < j1) sl[t[k]] = x[k];
  }
  __syncthreads();
  // the bucket's ids [id0, id0 + cnt) are all present exactly once: write them in order
  const u32 cnt = j1 - j0;
  constexpr u32 PER = 16u / sizeof(LT);
  uint4* dst = reinterpret_cast<uint4*>(labx + id0);  // id0 is a multiple of 2^PERM_SHIFT: 16-byte aligned
  for (u32 i = threadIdx.x; i < cnt / PER; i += blockDim.x) dst[i] = sl4[i];
  for (u32 i = (cnt / PER) * PER + threadIdx.x; i < cnt; i += blockDim.x) labx[id0 + i] = sl[i];
}


// STAGED: the labels were already moved to the stored order into labx (sentinel = out of
// range); otherwise they are read from labels[perm[u]] (or labels[u]) and written to labx.
// Label range: the LDS histograms hold the LR labels [lbase, lbase + LR); a label space
// wider than the LDS budget is counted in several launches, one per range, each node in
// the launch whose range holds its label (which gives its offset loc[u]).  The launch
// with lbase = 0 also flags invalid labels and writes labx; the others skip nodes with
// invalid labels.
template <bool WEIGHTED, class LT, bool STAGED = false>
__device__ __forceinline__ void node_priv_body(int n, const int32_t* __restrict__ labels, const int32_t* __restrict__ perm,
                                               const int32_t* __restrict__ rp, int L, int chunk, u32* __restrict__ HN,
                                               u32* __restrict__ HD, u32* __restrict__ loc, LT* __restrict__ labx,
                                               Ctl* __restrict__ ctl, int blk, int lbase, int LR, int lst = 1) {
  extern __shared__ u32 sh[];
  u32* hn = sh;
  u32* hd = WEIGHTED ? sh + LR : sh;
  __shared__ u32 s_bad;
  const int words = WEIGHTED ? 2 * LR : LR;
  for (int i = threadIdx.x; i < words; i += blockDim.x) sh[i] = 0;
  if (threadIdx.x == 0) s_bad = 0;
  __syncthreads();
  const bool first = lbase == 0;
  const long long u0 = (long long)blk * chunk;
  const long long u1 = min((long long)n, u0 + chunk);
  const int lane = threadIdx.x & 63;
  u32 bad = 0;
  for (long long ub = u0; ub < u1; ub += blockDim.x) {  // uniform trip count per wave
    const long long u = ub + threadIdx.x;
    const bool in = u < u1;
    int c;
    if (STAGED) {
      const u32 x = in ? (u32)labx[u * lst] : 0u;
      c = x == (u32)LabelT<LT>::SENTINEL ? -1 : (int)x;
    } else {
      c = in ? labels[perm ? perm[u] : u] : 0;
    }
    const bool valid = in && (u32)c < (u32)L;
    if (first && in && !valid) {
      bad = 1;
      loc[u] = SENT;
      if (labx && !STAGED) labx[u * lst] = LabelT<LT>::SENTINEL;
    }
    const int cl = c - lbase;
    const bool here = valid && (u32)cl < (u32)LR;
    const u32 w = here ? (WEIGHTED ? (u32)(rp[u + 1] - rp[u]) : 1u) : 0u;
    // Lanes with equal labels (common when the graph is stored in a locality order)
    // add to the LDS histogram through one leader lane; each lane's offset is the
    // leader's old value plus the weights of the group's lower lanes.
    bool pending = here;
    u32 old = 0;
    for (int round = 0; round < 4; ++round) {
      const u64 act = __ballot(pending);
      if (act == 0) break;
      const int leader = __ffsll((long long)act) - 1;
      const int lc = __shfl(cl, leader, 64);
      const bool mine = pending && cl == lc;
      const u64 grp = __ballot(mine);
      if (__popcll(grp) < 4) break;  // mixed labels: plain atomics below
      const u32 pw = mine ? w : 0u;
      const u32 incl = wave_incl_scan(pw);
      const u32 tot = __shfl(incl, 63, 64);
      u32 b = 0;
      if (lane == leader) {
        if (WEIGHTED) atomicAdd(&hn[lc], (u32)__popcll(grp));
        b = atomicAdd(&hd[lc], tot);
      }
      b = __shfl(b, leader, 64);
      if (mine) {
        old = b + incl - pw;
        pending = false;
      }
    }
    if (pending) {
      if (WEIGHTED) atomicAdd(&hn[cl], 1u);
      old = atomicAdd(&hd[cl], w);
    }
    if (here) loc[u] = old;
    if (first && valid && labx && !STAGED) labx[u * lst] = (LT)c;
  }
  if (bad) s_bad = 1;
  __syncthreads();
  const size_t row = (size_t)blk * (size_t)L + (size_t)lbase;
  for (int c = threadIdx.x; c < LR; c += blockDim.x) {
    HN[row + c] = hn[c];
    if (WEIGHTED) HD[row + c] = hd[c];
  }
  if (threadIdx.x == 0 && s_bad) atomicOr(&ctl->flags, F_LABEL);
}

// run_if != 0: the launch does nothing unless ctl->mode == run_if (the staging choice is
// made on the device, so both choices' kernels are enqueued and one of them returns).
template <bool WEIGHTED, class LT, bool STAGED = false>
__global__ __launch_bounds__(1024) void k_node_priv(int n, const int32_t* __restrict__ labels, const int32_t* __restrict__ perm,
                                                    const int32_t* __restrict__ rp, int L, int chunk, u32* __restrict__ HN,
                                                    u32* __restrict__ HD, u32* __restrict__ loc, LT* __restrict__ labx,
                                                    Ctl* __restrict__ ctl, int lbase, int LR, u32 run_if = 0) {
  if (run_if && ctl->mode != run_if) return;
  node_priv_body<WEIGHTED, LT, STAGED>(n, labels, perm, rp, L, chunk, HN, HD, loc, labx, ctl, blockIdx.x, lbase, LR);
}

// Node pass with global atomics (too many labels for LDS).  SZ[c] packs
// (count << 32) | weight sum; the returned old value gives the node's offset.
template <bool WEIGHTED, class LT, bool STAGED = false>
__global__ __launch_bounds__(256) void k_node_global(int n, const int32_t* __restrict__ labels, const int32_t* __restrict__ perm,
                                                     const int32_t* __restrict__ rp, int L, unsigned long long* __restrict__ SZ,
                                                     u32* __restrict__ loc, LT* __restrict__ labx, Ctl* __restrict__ ctl) {
  const int lane = threadIdx.x & 63;
  u32 bad = 0;
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (size_t ub = (size_t)blockIdx.x * blockDim.x; ub < (size_t)n; ub += stride) {  // uniform per wave
    const size_t u = ub + threadIdx.x;
    const bool in = u < (size_t)n;
    int c;
    if (STAGED) {
      const u32 x = in ? (u32)labx[u] : 0u;
      c = x == (u32)LabelT<LT>::SENTINEL ? -1 : (int)x;
    } else {
      c = in ? labels[perm ? perm[u] : u] : 0;
    }
    const bool valid = in && (u32)c < (u32)L;
    if (in && !valid) {
      bad = 1;
      loc[u] = SENT;
      if (labx && !STAGED) labx[u] = LabelT<LT>::SENTINEL;
    }
    const u32 w = valid ? (WEIGHTED ? (u32)(rp[u + 1] - rp[u]) : 1u) : 0u;
    // lanes with equal labels add through one leader (see k_node_priv)
    bool pending = valid;
    u32 old = 0;
    for (int round = 0; round < 4; ++round) {
      const u64 act = __ballot(pending);
      if (act == 0) break;
      const int leader = __ffsll((long long)act) - 1;
      const int lc = __shfl(c, leader, 64);
      const bool mine = pending && c == lc;
      const u64 grp = __ballot(mine);
      if (__popcll(grp) < 4) break;
      const u32 pw = mine ? w : 0u;
      const u32 incl = wave_incl_scan(pw);
      const u32 tot = __shfl(incl, 63, 64);
      u32 b = 0;
      if (lane == leader) b = (u32)atomicAdd(&SZ[lc], ((unsigned long long)__popcll(grp) << 32) | (unsigned long long)tot);
      b = __shfl(b, leader, 64);
      if (mine) {
        old = b + incl - pw;
        pending = false;
      }
    }
    if (pending) old = (u32)atomicAdd(&SZ[c], (1ull << 32) | (unsigned long long)w);
    if (valid) {
      loc[u] = old;
      if (labx && !STAGED) labx[u] = (LT)c;
    }
  }
  if (bad) atomicOr(&ctl->flags, F_LABEL);
}

// Plain label histogram (no slots): detected-partition sizes |c'| for the comparison,
// for the LR labels [lbase, lbase + LR) (one launch per range, as in the node pass; the
// launch with lbase = 0 flags invalid labels).
__global__ __launch_bounds__(1024) void k_hist_priv(int n, const int32_t* __restrict__ labels, int L, u32* __restrict__ HN,
                                                    Ctl* __restrict__ ctl, int lbase, int LR) {
  extern __shared__ u32 sh[];
  __shared__ u32 s_bad;
  for (int i = threadIdx.x; i < LR; i += blockDim.x) sh[i] = 0;
  if (threadIdx.x == 0) s_bad = 0;
  __syncthreads();
  u32 bad = 0;
  for (size_t u = (size_t)blockIdx.x * blockDim.x + threadIdx.x; u < (size_t)n; u += (size_t)gridDim.x * blockDim.x) {
    const int c = labels[u];
    if ((u32)c >= (u32)L) {
      bad = 1;
      continue;
    }
    const int cl = c - lbase;
    if ((u32)cl < (u32)LR) atomicAdd(&sh[cl], 1u);
  }
  if (bad && lbase == 0) s_bad = 1;
  __syncthreads();
  const size_t row = (size_t)blockIdx.x * (size_t)L + (size_t)lbase;
  for (int c = threadIdx.x; c < LR; c += blockDim.x) HN[row + c] = sh[c];
  if (threadIdx.x == 0 && s_bad) atomicOr(&ctl->flags, F_LABEL);
}

__global__ __launch_bounds__(256) void k_hist_global(int n, const int32_t* __restrict__ labels, int L, u32* __restrict__ cnt,
                                                     Ctl* __restrict__ ctl) {
  u32 bad = 0;
  for (size_t u = (size_t)blockIdx.x * blockDim.x + threadIdx.x; u < (size_t)n; u += (size_t)gridDim.x * blockDim.x) {
    int c = labels[u];
    if ((u32)c >= (u32)L) { bad = 1; continue; }
    atomicAdd(&cnt[c], 1u);
  }
  if (bad) atomicOr(&ctl->flags, F_LABEL);
}

// Column pass over the per-workgroup histograms: totals per label, and (SCAN) the
// exclusive prefix over workgroups written back into the prefix matrix PM.
template <bool WEIGHTED, bool SCAN>
__device__ __forceinline__ void colscan_body(int W, int L, u32* __restrict__ HN, u32* __restrict__ HD, u32* __restrict__ N,
                                             u32* __restrict__ D, int c) {
  u32* PM = WEIGHTED ? HD : HN;
  u32 sn = 0, sd = 0;
  int w = 0;
  for (; w + 8 <= W; w += 8) {
    u32 xn[8], xd[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      xn[k] = HN[(size_t)(w + k) * L + c];
      xd[k] = WEIGHTED ? HD[(size_t)(w + k) * L + c] : xn[k];
    }
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      if (SCAN) PM[(size_t)(w + k) * L + c] = sd;
      sn += xn[k];
      sd += xd[k];
    }
  }
  for (; w < W; ++w) {
    u32 xn = HN[(size_t)w * L + c];
    u32 xd = WEIGHTED ? HD[(size_t)w * L + c] : xn;
    if (SCAN) PM[(size_t)w * L + c] = sd;
    sn += xn;
    sd += xd;
  }
  N[c] = sn;
  if (D) D[c] = sd;
}

// The same over many rows: a workgroup takes 64 labels (one per lane, so every row read
// is coalesced) and 16 groups of consecutive rows.  Each group sums its rows, the groups'
// sums are combined in LDS, and with SCAN each group writes its rows' prefixes starting
// from the sum of the groups before it.
constexpr int CS_LABELS = 64;
constexpr int CS_GROUPS = 16;
// zero64 (optional): one 64-bit word per label cleared on the way (the run cursors).
template <bool WEIGHTED, bool SCAN>
__global__ __launch_bounds__(CS_LABELS * CS_GROUPS) void k_colscan(int W, int L, u32* __restrict__ HN,
                                                                   u32* __restrict__ HD, u32* __restrict__ N,
                                                                   u32* __restrict__ D,
                                                                   unsigned long long* __restrict__ zero64 = nullptr,
                                                                   const Ctl* __restrict__ gate = nullptr, u32 run_if = 0) {
  if (gate && gate->mode != run_if) return;  // see k_node_priv
  __shared__ u32 s_n[CS_GROUPS][CS_LABELS], s_d[CS_GROUPS][CS_LABELS];
  const int lane = threadIdx.x % CS_LABELS, grp = threadIdx.x / CS_LABELS;
  const int c = blockIdx.x * CS_LABELS + lane;
  const int per = (W + CS_GROUPS - 1) / CS_GROUPS;
  const int w0 = min(W, grp * per), w1 = min(W, w0 + per);
  u32* PM = WEIGHTED ? HD : HN;
  u32 sn = 0, sd = 0;
  if (c < L) {
    for (int w = w0; w < w1; ++w) {
      const u32 xn = HN[(size_t)w * L + c];
      sn += xn;
      sd += WEIGHTED ? HD[(size_t)w * L + c] : xn;
    }
  }
  s_n[grp][lane] = sn;
  s_d[grp][lane] = sd;
  __syncthreads();
  if (c >= L) return;
  if (SCAN) {
    u32 run = 0;
    for (int i = 0; i < grp; ++i) run += s_d[i][lane];
    for (int w = w0; w < w1; ++w) {
      const size_t at = (size_t)w * L + c;
      const u32 x = WEIGHTED ? HD[at] : HN[at];
      PM[at] = run;
      run += x;
    }
  }
  if (grp == 0) {
    u32 tn = 0, td = 0;
    for (int i = 0; i < CS_GROUPS; ++i) {
      tn += s_n[i][lane];
      td += s_d[i][lane];
    }
    N[c] = tn;
    if (D) D[c] = td;
    if (zero64) zero64[c] = 0ull;
  }
}

// Column-blocked node pass: adds the histogram rows of the dense buckets (rows[0,
// ctl->dense_rows), written by k_perm_apply_count) to N and D, and clears the 64-bit run
// cursors.  Integer sums, so the order of the row list does not matter.
// It also chooses how the call stages neighbour labels (Ctl::mode): through the row-major
// copy when the stored-order labels change at least `rows_from` times (a partition that
// does not follow the stored order), else through the column blocks.
__global__ __launch_bounds__(256) void k_colscan_rows(int L, const u32* __restrict__ HN, const u32* __restrict__ HD,
                                                      const u32* __restrict__ rows, Ctl* __restrict__ ctl,
                                                      u32* __restrict__ N, u32* __restrict__ D,
                                                      unsigned long long* __restrict__ zero64, u32 rows_from) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  const u32 mode = ctl->changes >= rows_from ? STAGE_ROWS : STAGE_BLOCKS;  // every thread reads the final count
  if (c == 0) ctl->mode = mode;
  if (c >= L) return;
  if (mode == STAGE_ROWS) {
    zero64[c] = 0ull;  // N and D come from the row-major node pass (k_colscan after k_node_priv)
    return;
  }
  const u32 nd = ctl->dense_rows;
  if (nd) {
    u32 sn = 0, sd = 0;
    for (u32 i = 0; i < nd; ++i) {
      const size_t at = (size_t)rows[i] * (size_t)L + (size_t)c;
      sn += HN[at];
      sd += HD[at];
    }
    N[c] += sn;
    D[c] += sd;
  }
  zero64[c] = 0ull;
}

__global__ void k_unpack(int L, const unsigned long long* __restrict__ SZ, u32* __restrict__ N, u32* __restrict__ D) {
  for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < L; c += gridDim.x * blockDim.x) {
    unsigned long long v = SZ[c];
    N[c] = (u32)(v >> 32);
    if (D) D[c] = (u32)v;
  }
}

// ---------------------------------------------------------------------------
// Segment starts (exclusive scan of the weights D) and the work order of the
// non-empty groups: by decreasing floor(log2 D), so the largest groups start first.
__device__ __forceinline__ int size_bucket(u32 x) { return x ? 32 - __clz(x) : 0; }
// Groups whose weight (segment length bound) is below GW_SPLIT = 2^(GW_SPLIT_BUCKET - 1)
// come last in the order; the comparison counts them one per wave (k_groups_wave).
constexpr int GW_SPLIT_BUCKET = 12;
constexpr u32 GW_SPLIT = 1u << (GW_SPLIT_BUCKET - 1);  // 2048

// Values of labels c0 .. c0+15 (0 past L): 16-byte loads when all 16 exist (c0 is a
// multiple of 16 and the arrays 16-byte aligned), else one guarded load per label.
__device__ __forceinline__ void load_labels16(int c0, int L, const u32* __restrict__ N, const u32* __restrict__ D,
                                              u32 (&d)[16], u32 (&nn)[16]) {
  typedef u32 v4u __attribute__((ext_vector_type(4)));
  if (c0 + 16 <= L) {
    const v4u* dv = reinterpret_cast<const v4u*>(D + c0);
    const v4u* nv = reinterpret_cast<const v4u*>(N + c0);
    v4u a[4], b[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      a[i] = dv[i];
      b[i] = nv[i];
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      d[4 * i] = a[i].x; d[4 * i + 1] = a[i].y; d[4 * i + 2] = a[i].z; d[4 * i + 3] = a[i].w;
      nn[4 * i] = b[i].x; nn[4 * i + 1] = b[i].y; nn[4 * i + 2] = b[i].z; nn[4 * i + 3] = b[i].w;
    }
  } else {
#pragma unroll
    for (int k = 0; k < 16; ++k) {
      const int c = c0 + k;
      d[k] = c < L ? D[c] : 0u;
      nn[k] = c < L ? N[c] : 0u;
    }
  }
}

// One workgroup of 1024 threads; thread t takes SO_PER consecutive labels of each pass
// of 1024 * SO_PER, with all of their loads issued before the first use.
constexpr int SO_PER = 16;  // load_labels16
__device__ void scan_order_body(int L, const u32* __restrict__ N, const u32* __restrict__ D, u32* __restrict__ start,
                                u32* __restrict__ order, Ctl* __restrict__ ctl) {
  __shared__ u32 s_wtot[16];
  __shared__ u32 s_carry;
  __shared__ u32 s_bcnt[33];
  __shared__ u32 s_boff[33];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  if (tid < 33) s_bcnt[tid] = 0;
  if (tid == 0) s_carry = 0;
  __syncthreads();
  for (int base = 0; base < L; base += 1024 * SO_PER) {
    const int c0 = base + tid * SO_PER;
    u32 d[SO_PER], nn[SO_PER];
    load_labels16(c0, L, N, D, d, nn);
    u32 sum = 0;
#pragma unroll
    for (int k = 0; k < SO_PER; ++k) {
      sum += d[k];
      if (nn[k] > 0) atomicAdd(&s_bcnt[size_bucket(d[k])], 1u);
    }
    const u32 incl = wave_incl_scan(sum);
    if (lane == 63) s_wtot[wv] = incl;
    __syncthreads();
    u32 run = s_carry + incl - sum;
    for (int i = 0; i < wv; ++i) run += s_wtot[i];
#pragma unroll
    for (int k = 0; k < SO_PER; ++k) {
      if (c0 + k < L) start[c0 + k] = run;
      run += d[k];
    }
    __syncthreads();
    if (tid == 0) {
      u32 t = s_carry;
      for (int i = 0; i < 16; ++i) t += s_wtot[i];
      s_carry = t;
    }
    __syncthreads();
  }
  if (tid == 0) {
    u32 off = 0;
    for (int b = 32; b >= 0; --b) { s_boff[b] = off; off += s_bcnt[b]; }
    ctl->K = off;
    ctl->kbig = s_boff[GW_SPLIT_BUCKET - 1];  // groups in buckets >= GW_SPLIT_BUCKET
  }
  __syncthreads();
  for (int base = 0; base < L; base += 1024 * SO_PER) {
    const int c0 = base + tid * SO_PER;
    u32 d[SO_PER], nn[SO_PER];
    load_labels16(c0, L, N, D, d, nn);
#pragma unroll
    for (int k = 0; k < SO_PER; ++k) {
      if (nn[k] > 0) order[atomicAdd(&s_boff[size_bucket(d[k])], 1u)] = (u32)(c0 + k);
    }
  }
}

__global__ __launch_bounds__(1024) void k_scan_order(int L, const u32* __restrict__ N, const u32* __restrict__ D,
                                                     u32* __restrict__ start, u32* __restrict__ order, Ctl* __restrict__ ctl) {
  scan_order_body(L, N, D, start, order, ctl);
}

// ---------------------------------------------------------------------------
// Edge pass: for every stored entry (u, v) write label[v] into the segment of
// community label[u] at start[c_u] + (offset of u) + (position of v in u's row).
// A workgroup takes 256 consecutive rows; their entries are contiguous in col_idx and
// are walked by all threads in order (coalesced); the owning row of an entry is found
// by binary search over the 256 row starts staged in LDS.
constexpr int GROWS = 256;
template <bool PRIV, class LT, bool WT>
__device__ __forceinline__ void gather_rows(long long r0, int n, const int32_t* __restrict__ rp, const int32_t* __restrict__ col,
                                            const LT* __restrict__ labx, int L, int chunk, const u32* __restrict__ PM,
                                            const u32* __restrict__ start, const u32* __restrict__ loc, LT* __restrict__ CB,
                                            const float* __restrict__ w, float* __restrict__ CW, int* s_rs, u32* s_base) {
  const int tid = threadIdx.x;
  const int rows = (int)min((long long)GROWS, (long long)n - r0);
  if (tid < rows) {
    long long u = r0 + tid;
    s_rs[tid] = rp[u];
    const LT c = labx[u];
    const u32 lu = loc[u];
    u32 base = SENT;
    if (c != LabelT<LT>::SENTINEL && lu != SENT) {
      base = start[c] + lu;
      if (PRIV) base += PM[(size_t)(u / chunk) * L + c];
    }
    s_base[tid] = base;
  }
  if (tid == 0) s_rs[rows] = rp[r0 + rows];
  __syncthreads();
  const int e0 = s_rs[0], e1 = s_rs[rows];
  for (int e = e0 + tid; e < e1; e += GROWS) {
    int lo = 0, hi = rows - 1;  // last row r with s_rs[r] <= e
    while (lo < hi) {
      int mid = (lo + hi + 1) >> 1;
      if (s_rs[mid] <= e) lo = mid; else hi = mid - 1;
    }
    const u32 base = s_base[lo];
    if (base == SENT) continue;
    CB[base + (u32)(e - s_rs[lo])] = labx[col[e]];
    if (WT) CW[base + (u32)(e - s_rs[lo])] = w[e];
  }
}

// Tiles of GROWS rows.  With one workgroup per tile (grid of 8 * ceil(tiles / 8)),
// workgroup b runs on XCD b % 8 and takes tile (b % 8) * ceil(tiles / 8) + b / 8: each
// XCD walks its own eighth of the rows in order, so the labels that neighbouring rows
// share stay in its L2 (the 100M-node graph's edge pass: 7.63 -> 7.40 ms).  A smaller
// grid takes the tiles in turn (grid-stride).  gate (optional): the launch does nothing
// unless gate->mode == STAGE_ROWS (a column-blocked graph scored through its row-major
// copy; see k_colscan_rows).
template <bool PRIV, class LT, bool WT>
__global__ __launch_bounds__(GROWS) void k_gather(int n, const int32_t* __restrict__ rp, const int32_t* __restrict__ col,
                                                  const LT* __restrict__ labx, int L, int chunk, const u32* __restrict__ PM,
                                                  const u32* __restrict__ start, const u32* __restrict__ loc,
                                                  LT* __restrict__ CB, const float* __restrict__ w, float* __restrict__ CW,
                                                  const Ctl* __restrict__ gate = nullptr) {
  __shared__ int s_rs[GROWS + 1];
  __shared__ u32 s_base[GROWS];
  if (gate && gate->mode != STAGE_ROWS) return;
  const long long tiles = ((long long)n + GROWS - 1) / GROWS;
  const long long per = (tiles + 7) / 8;
  if (gridDim.x >= 8 * per) {
    const long long t = (long long)(blockIdx.x % 8u) * per + blockIdx.x / 8u;
    if (t < tiles) gather_rows<PRIV, LT, WT>(t * GROWS, n, rp, col, labx, L, chunk, PM, start, loc, CB, w, CW, s_rs, s_base);
    return;
  }
  for (long long t = blockIdx.x; t < tiles; t += gridDim.x) {
    gather_rows<PRIV, LT, WT>(t * GROWS, n, rp, col, labx, L, chunk, PM, start, loc, CB, w, CW, s_rs, s_base);
    __syncthreads();  // the next tile's row starts replace this one's
  }
}

// Edge pass over a column-blocked graph.  Workgroup i runs on XCD i % 8 (workgroups
// are handed to the XCDs in turn) and takes entries of column block y = i % 8, so every
// neighbour label an XCD reads lies in the span of ids its own L2 holds.  Two kinds of
// tile share the work of block y: own-span tiles take rows of span y itself (most
// entries: a row's community mostly lies in its own span; the labels of ids near the
// tile are staged in LDS), far tiles take the block's entries in the rows of the other
// spans as a list of (row, neighbour) pairs (under one entry per row, so per-row
// headers would cost more than the entries).  In a tile, rows with equal labels that
// follow each other form a run; one atomic add on the community's cursor gives the run
// consecutive places in the community's segment, and each entry goes to run start +
// its index in the run.
constexpr int BT_THREADS = 256;
constexpr int BT_UNROLL = 8;     // entries in flight per thread
constexpr int BT_HALO = 1024;    // OWN tiles keep labels of ids within this distance of their rows in LDS
constexpr int BT_RPT = 2;                        // rows per thread in own-span tiles
constexpr int BT_ROWS = BT_THREADS * BT_RPT;     // rows per own-span tile
// Far entries per thread: few, since each is a random label read; weighted entries
// carry a weight load as well and run best with fewer still.
constexpr int FT_EPT = 4;
constexpr int FT_EPT_W = 2;
constexpr int FT_ENT = BT_THREADS * FT_EPT;      // far entries per tile
constexpr int FT_ENT_W = BT_THREADS * FT_EPT_W;  // far entries per tile, weighted graphs
constexpr int OWN_BUF = 1024;  // entries of another label an own-span tile keeps in LDS (compact staging)
constexpr int OWN_BUF_W = 512;  // the same for weighted graphs (with weights and run sums: six workgroups per CU)

// Far entries of column block y: colb/rowb ranges [b[y][0], b[y][1]) (rows before span y)
// and [b[y][2], b[y][3]) (rows after it), row-major.
struct FarTable {
  u32 b[COL_BLOCKS][4];
};

template <class LT, bool WT = false>
struct GatherLds {
  static constexpr int PER = 16 / (int)sizeof(LT);             // labels per 16-byte word
  static constexpr int WINV = (BT_ROWS + 2 * BT_HALO) / PER + 1;  // 16-byte words of the label window
  static constexpr int RUN_WORDS = (4 * (BT_ROWS + 1) + 3) & ~3;  // four per-run arrays, padded to 16 bytes
  static constexpr int BUF = sizeof(LT) == 2 ? (WT ? OWN_BUF_W : OWN_BUF) : 0;  // compact staging buffer (16-bit labels)
  static constexpr int WBUF = WT ? BUF : 0;                        // the buffered entries' weights
  static constexpr int ISUM = WT ? 4 * BT_ROWS : 0;                // per run: own-label weight sum, two u64
  static constexpr int OWN = RUN_WORDS + 4 * WINV + BUF + WBUF + ISUM;
  static constexpr int FAR = 3 * (FT_ENT + 1);
  static constexpr int WORDS = OWN > FAR ? OWN : FAR;
};

// Block-wide run numbering: `heads` marks (bit j) the thread's items that start a run.
// Returns the number of heads before this thread's items; *nruns gets the total.
__device__ __forceinline__ u32 runs_before(u32 heads, u32* s_w, u32* nruns) {
  const u32 nh = (u32)__popc(heads);
  const u32 incl = wave_incl_scan(nh);
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 63) s_w[w] = incl;
  __syncthreads();
  u32 q = incl - nh, tot = 0;
  for (int i = 0; i < BT_THREADS / 64; ++i) {
    if (i < w) q += s_w[i];
    tot += s_w[i];
  }
  *nruns = tot;
  return q;
}

// Gives every run (label c = s_lab[r], entries s_first[r] .. s_first[r+1]) consecutive
// places in segment c: s_lab[r] becomes the place of its first entry, or SENT.
template <class LT>
__device__ __forceinline__ void claim_runs(u32 nruns, const u32* s_first, u32* s_lab, const u32* __restrict__ start,
                                           const u32* __restrict__ D, u32* __restrict__ cursor, Ctl* __restrict__ ctl) {
  for (u32 r = threadIdx.x; r < nruns; r += BT_THREADS) {
    const u32 c = s_lab[r];
    const u32 tot = s_first[r + 1] - s_first[r];
    u32 base = SENT;
    if (c != (u32)LabelT<LT>::SENTINEL && tot > 0) {
      const u32 old = atomicAdd(&cursor[c], tot);
      if (old + tot <= D[c]) base = start[c] + old;  // < 2^31, so never the SENT marker
      else atomicOr(&ctl->flags, F_SEGMENT);  // never expected: the block counts disagree with the degrees
    }
    s_lab[r] = base;
  }
}

// Compact staging (unweighted graphs): an entry whose neighbour carries the row's own label
// adds only to 2|E_c^in| and is not staged.  Run r of label c (entries s_first[r] ..
// s_first[r+1], s_cnt[r] of them with another label) adds (intra << 32) | inter to
// cur64[c] with one atomic: the low word is the segment cursor, the high word the intra
// count.  s_base[r] gets the place of the run's first staged entry, or SENT; s_cnt[r]
// is reset so that it can hand out places inside the run.
template <class LT>
__device__ __forceinline__ void claim_runs_compact(u32 nruns, const u32* s_first, const u32* s_lab, u32* s_cnt,
                                                   u32* s_base, const u32* __restrict__ start, const u32* __restrict__ D,
                                                   unsigned long long* __restrict__ cur64, Ctl* __restrict__ ctl) {
  for (u32 r = threadIdx.x; r < nruns; r += BT_THREADS) {
    const u32 c = s_lab[r];
    const u32 tot = s_first[r + 1] - s_first[r];
    const u32 inter = s_cnt[r];
    u32 base = SENT;
    if (c != (u32)LabelT<LT>::SENTINEL && tot > 0) {
      const unsigned long long old = atomicAdd(&cur64[c], ((unsigned long long)(tot - inter) << 32) | inter);
      const u32 lo = (u32)old;
      if (lo + inter <= D[c]) base = start[c] + lo;  // < 2^31, so never the SENT marker
      else atomicOr(&ctl->flags, F_SEGMENT);  // never expected: the block counts disagree with the degrees
    }
    s_base[r] = base;
    s_cnt[r] = 0;
  }
}

// Own-span tile t of block y: rows [s0 + t*BT_ROWS, ...) of span y, their block-y entries.
// Staging is compact (claim_runs_compact): a first pass over the tile's entries counts
// each run's entries of another label, the runs claim their places, and those entries
// are staged (from an LDS buffer, or by a second pass when it overflows).  WT: the graph
// is weighted: a staged entry's weight goes to CW beside its label, and each run's
// own-label weights are summed exactly (x 2^55, as WeightSum) and added to IWacc[c] (two
// u64 words per community, low word first, the carry added to the high word).
template <class LT, bool WT>
__device__ void gather_own_tile(u32 y, u32 t, int n, int span, const u32* __restrict__ RPB,
                                const int32_t* __restrict__ colb, const LT* __restrict__ labx,
                                const u32* __restrict__ start, const u32* __restrict__ D, u32* __restrict__ cursor,
                                Ctl* __restrict__ ctl, LT* __restrict__ CB, const float* __restrict__ wb,
                                float* __restrict__ CW, unsigned long long* __restrict__ IWacc, u32* lds, u32* s_w) {
  using LL = GatherLds<LT, WT>;
  constexpr int PER = LL::PER;
  constexpr int WIT = (LL::WINV + BT_THREADS - 1) / BT_THREADS;
  u32* s_re = lds;                   // staged row starts, then first entry of run q (tile-relative)
  u32* s_rl = lds + BT_ROWS + 1;     // staged row labels, then label of run q
  u32* s_cnt = lds + 2 * (BT_ROWS + 1);   // entries of run q with another label
  u32* s_base = lds + 3 * (BT_ROWS + 1);  // place of run q's first staged entry
  uint4* s_win = reinterpret_cast<uint4*>(lds + LL::RUN_WORDS);  // labels of ids [w0, w1)
  // WT: own-label weight sum of run q (low, high words)
  unsigned long long* s_ilo =
      reinterpret_cast<unsigned long long*>(lds + LL::RUN_WORDS + 4 * LL::WINV + LL::BUF + LL::WBUF);
  unsigned long long* s_ihi = s_ilo + BT_ROWS;
  const long long s0 = min((long long)n, (long long)y * span), s1 = min((long long)n, s0 + span);
  const long long r0 = s0 + (long long)t * BT_ROWS, r1 = min(s1, r0 + BT_ROWS);
  if (r0 >= r1) return;
  const u32* rpb = RPB + (size_t)y * ((size_t)n + 1);
  const int rows = (int)(r1 - r0);
  const u32 e0 = rpb[r0], e1 = rpb[r1];
  if (e0 == e1) return;
  const int tid = threadIdx.x;
  // Stage the tile's row starts and labels and the label window (coalesced; every load
  // is issued before the first one is used), then each thread takes BT_RPT rows.
  const long long w0 = (max(0ll, r0 - BT_HALO) / PER) * PER;
  const long long w1 = max(w0, (min((long long)n, r1 + BT_HALO) / PER) * PER);
  {
    u32 ra[BT_RPT], rl[BT_RPT];
#pragma unroll
    for (int j = 0; j < BT_RPT; ++j) {
      const int r = min(tid + j * BT_THREADS, rows - 1);
      ra[j] = rpb[r0 + r];
      rl[j] = (u32)labx[r0 + r];
    }
    // a native vector type: an array of HIP's uint4 class is kept in scratch memory
    typedef u32 v4u __attribute__((ext_vector_type(4)));
    const v4u* src = reinterpret_cast<const v4u*>(labx + w0);
    v4u* s_winv = reinterpret_cast<v4u*>(s_win);
    const int nv = (int)((w1 - w0) / PER);
    v4u wv[WIT];
    if (nv > 0) {  // uniform; every load unconditional (clamped)
#pragma unroll
      for (int j = 0; j < WIT; ++j) wv[j] = src[min(tid + j * BT_THREADS, nv - 1)];
    }
#pragma unroll
    for (int j = 0; j < BT_RPT; ++j) {
      const int r = tid + j * BT_THREADS;
      if (r < rows) {
        s_re[r] = ra[j] - e0;
        s_rl[r] = rl[j];
      }
    }
#pragma unroll
    for (int j = 0; j < WIT; ++j) {
      const int i = tid + j * BT_THREADS;
      if (i < nv) s_winv[i] = wv[j];
    }
  }
  __syncthreads();
  u32 lab[BT_RPT], beg[BT_RPT];
  u32 heads = 0;
  const int rb = BT_RPT * tid;
  u32 prev = rb > 0 && rb - 1 < rows ? s_rl[rb - 1] : 0xFFFFFFFFu;
#pragma unroll
  for (int j = 0; j < BT_RPT; ++j) {
    const int r = rb + j;
    lab[j] = r < rows ? s_rl[r] : 0u;
    beg[j] = r < rows ? s_re[r] : 0u;
    if (r < rows && (r == 0 || lab[j] != prev)) heads |= 1u << j;
    prev = lab[j];
  }
  u32 nruns;
  u32 q = runs_before(heads, s_w, &nruns);  // its barrier also ends the reads of staged rows
#pragma unroll
  for (int j = 0; j < BT_RPT; ++j) {
    if (heads & (1u << j)) {
      s_re[q] = beg[j];
      s_rl[q] = lab[j];
      ++q;
    }
  }
  if (tid == 0) {
    s_re[nruns] = e1 - e0;
    s_base[BT_ROWS] = 0;  // compact: count of buffered entries
  }
  for (u32 r = tid; r < nruns; r += BT_THREADS) {
    s_cnt[r] = 0;
    if (WT) {
      s_ilo[r] = 0ull;
      s_ihi[r] = 0ull;
    }
  }
  __syncthreads();
  const int32_t* cb = colb + e0;
  const u32 ne = e1 - e0;
  // f(e, run, x, w) for the BT_UNROLL entries e = eb + u*BT_THREADS of each chunk (e < ne);
  // w is the entry's weight (WT) or 0
  auto for_entries = [&](auto&& f) {
    for (u32 eb = tid; eb < ne; eb += BT_THREADS * BT_UNROLL) {
      int v[BT_UNROLL];
      float wt[BT_UNROLL];
      u32 run[BT_UNROLL];
#pragma unroll
      for (int u = 0; u < BT_UNROLL; ++u) v[u] = cb[min(eb + (u32)(u * BT_THREADS), ne - 1u)];  // in bounds; masked below
#pragma unroll
      for (int u = 0; u < BT_UNROLL; ++u)  // loaded with the ids, so their latency overlaps the run search
        wt[u] = WT ? wb[e0 + min(eb + (u32)(u * BT_THREADS), ne - 1u)] : 0.0f;
#pragma unroll
      for (int u = 0; u < BT_UNROLL; ++u) {
        const u32 e = eb + (u32)(u * BT_THREADS);
        u32 lo = 0, hi = nruns - 1;  // last run r with s_re[r] <= e
        while (lo < hi) {
          const u32 mid = (lo + hi + 1) >> 1;
          if (s_re[mid] <= e) lo = mid; else hi = mid - 1;
        }
        run[u] = lo;
      }
      LT x[BT_UNROLL];
#pragma unroll
      for (int u = 0; u < BT_UNROLL; ++u) {
        const u32 off = (u32)((long long)v[u] - w0);
        x[u] = off < (u32)(w1 - w0) ? reinterpret_cast<const LT*>(s_win)[off] : labx[v[u]];
      }
#pragma unroll
      for (int u = 0; u < BT_UNROLL; ++u) {
        const u32 e = eb + (u32)(u * BT_THREADS);
        if (e < ne) f(e, run[u], x[u], wt[u]);
      }
    }
  };
  // Pass 1: count each run's entries of another label and keep them, (run << 16) | label
  // (and their weights, WT), in the LDS buffer; slots and counts are taken once per wave.
  u32* s_buf = lds + LL::RUN_WORDS + 4 * LL::WINV;
  float* s_wbuf = reinterpret_cast<float*>(s_buf + LL::BUF);
  u32* s_nbuf = s_base + BT_ROWS;  // unused by runs (nruns <= BT_ROWS)
  const int lane = tid & 63;
  const u64 below = lane ? (~0ull >> (64 - lane)) : 0ull;
  // WT: a thread meets its entries in increasing order, so runs in increasing order: it
  // sums the own-label weights of its current run and adds them to the run's LDS sum
  // when the run changes (64-bit atomics, the low word's carry added to the high word)
  u32 wrun = 0xFFFFFFFFu;
  WeightSum wacc;
  auto wflush = [&]() {
    if (wrun != 0xFFFFFFFFu) {
      const unsigned long long old = atomicAdd(&s_ilo[wrun], (unsigned long long)wacc.lo);
      const unsigned long long hi = wacc.hi + (old + wacc.lo < old ? 1ull : 0ull);
      if (hi) atomicAdd(&s_ihi[wrun], hi);
    }
  };
  for_entries([&](u32, u32 r, LT x, float w) {
    const bool inter = (u32)x != s_rl[r];
    if (WT && !inter) {
      if (r != wrun) {
        wflush();
        wrun = r;
        wacc = WeightSum();
      }
      u64 vlo, vhi;
      WeightSum::split(w, vlo, vhi);
      wacc.add(vlo, vhi);
    }
    const u64 m = __ballot(inter);
    if (m == 0) return;
    const int lead = __ffsll((long long)m) - 1;
    const u32 rl = __shfl(r, lead, 64);
    const u64 ms = __ballot(inter && r == rl);
    u32 slot0 = 0;
    if (lane == lead) {
      slot0 = atomicAdd(s_nbuf, (u32)__popcll(m));
      atomicAdd(&s_cnt[rl], (u32)__popcll(ms));
    }
    slot0 = __shfl(slot0, lead, 64);
    if (inter) {
      const u32 slot = slot0 + (u32)__popcll(m & below);
      if (slot < (u32)LL::BUF) {
        s_buf[slot] = (r << 16) | (u32)x;
        if (WT) s_wbuf[slot] = w;
      }
      if (r != rl) atomicAdd(&s_cnt[r], 1u);
    }
  });
  if (WT) wflush();
  __syncthreads();
  claim_runs_compact<LT>(nruns, s_re, s_rl, s_cnt, s_base, start, D, reinterpret_cast<unsigned long long*>(cursor), ctl);
  if (WT) {
    // each run's own-label weights join its community's sum
    for (u32 r = tid; r < nruns; r += BT_THREADS) {
      const unsigned long long lo = s_ilo[r], hi = s_ihi[r];
      const u32 c = s_rl[r];
      if ((lo | hi) && c != (u32)LabelT<LT>::SENTINEL) {
        const unsigned long long old = atomicAdd(&IWacc[2 * (size_t)c], lo);
        const unsigned long long h = hi + (old + lo < old ? 1ull : 0ull);
        if (h) atomicAdd(&IWacc[2 * (size_t)c + 1], h);
      }
    }
  }
  __syncthreads();
  const u32 nb = *s_nbuf;
  if (nb <= (u32)LL::BUF) {
    // write the buffer out: each wave takes consecutive places per run (coalesced)
    for (u32 k = tid; k < nb; k += BT_THREADS) {
      const u32 ent = s_buf[k];
      const u32 r = ent >> 16;
      const u64 act = __ballot(true);
      const int lead = __ffsll((long long)act) - 1;
      const u32 rl = __shfl(r, lead, 64);
      const u64 ms = __ballot(r == rl);
      u32 p0 = 0;
      if (lane == lead) p0 = atomicAdd(&s_cnt[rl], (u32)__popcll(ms));
      p0 = __shfl(p0, lead, 64);
      const u32 rank = r == rl ? p0 + (u32)__popcll(ms & below) : atomicAdd(&s_cnt[r], 1u);
      const u32 base = s_base[r];
      if (base != SENT) {
        CB[base + rank] = (LT)(ent & 0xFFFFu);
        if (WT) CW[base + rank] = s_wbuf[k];
      }
    }
  } else {
    // buffer overflow (or 32-bit labels): classify the tile's entries again
    for_entries([&](u32, u32 r, LT x, float w) {
      const u32 base = s_base[r];
      if ((u32)x != s_rl[r] && base != SENT) {
        const u32 rank = atomicAdd(&s_cnt[r], 1u);
        CB[base + rank] = x;
        if (WT) CW[base + rank] = w;
      }
    });
  }
}

// Far tile t of block y: FT_ENT (weighted: FT_ENT_W) consecutive entries of the block's
// far ranges.
template <class LT, bool WT>
__device__ void gather_far_tile(u32 y, u32 t, const FarTable& ft, const int32_t* __restrict__ colb,
                                const int32_t* __restrict__ rowb, const LT* __restrict__ labx,
                                const u32* __restrict__ start, const u32* __restrict__ D, u32* __restrict__ cursor,
                                Ctl* __restrict__ ctl, LT* __restrict__ CB, const float* __restrict__ wb,
                                float* __restrict__ CW, u32* lds, u32* s_w) {
  constexpr int EPT = WT ? FT_EPT_W : FT_EPT;
  constexpr u32 ENT = BT_THREADS * EPT;
  u32* s_rf = lds;                     // first entry of run q (tile-relative); s_rf[nruns] = entry count
  u32* s_rb = lds + ENT + 1;        // staged row labels, then label of run q, then its segment place
  u32* s_cnt = lds + 2 * (ENT + 1);  // compact: entries of run q with another label
  const u32 b0 = ft.b[y][0], b1 = ft.b[y][1], b2 = ft.b[y][2], b3 = ft.b[y][3];
  const u32 t1 = (b1 - b0 + ENT - 1) / ENT;
  u32 e0, e1;
  if (t < t1) {
    e0 = b0 + t * ENT;
    e1 = min(b1, e0 + ENT);
  } else {
    e0 = b2 + (t - t1) * ENT;
    if (e0 >= b3) return;
    e1 = min(b3, e0 + ENT);
  }
  const u32 ne = e1 - e0;
  const int tid = threadIdx.x;
  const u32 i0 = (u32)tid * EPT;  // this thread's entries i0 .. i0+EPT-1 (tile-relative)
  LT x[EPT];
  u32 lab[EPT];
  float wt[EPT];
#pragma unroll
  for (int j = 0; j < EPT; ++j) {
    const u32 e = e0 + min(i0 + (u32)j, ne - 1u);  // in bounds; entries past ne are masked below
    x[j] = labx[colb[e]];  // the neighbour labels are loaded now and used after the runs are placed
    lab[j] = (u32)labx[rowb[e]];
    if (WT) wt[j] = wb[e];
  }
#pragma unroll
  for (int j = 0; j < EPT; ++j)
    if (i0 + (u32)j < ne) s_rb[i0 + j] = lab[j];
  __syncthreads();
  u32 prev = (i0 > 0 && i0 - 1 < ne) ? s_rb[i0 - 1] : 0xFFFFFFFFu;
  u32 heads = 0;
#pragma unroll
  for (int j = 0; j < EPT; ++j) {
    const u32 i = i0 + (u32)j;
    if (i < ne && (i == 0 || lab[j] != prev)) heads |= 1u << j;
    prev = lab[j];
  }
  u32 nruns;
  const u32 q0 = runs_before(heads, s_w, &nruns);  // its barrier also ends the reads of staged labels
  {
    u32 q = q0;
#pragma unroll
    for (int j = 0; j < EPT; ++j) {
      if (heads & (1u << j)) {
        s_rf[q] = i0 + (u32)j;
        s_rb[q] = lab[j];
        ++q;
      }
    }
  }
  if (tid == 0) s_rf[nruns] = ne;
  if (!WT)
    for (u32 r = tid; r < nruns; r += BT_THREADS) s_cnt[r] = 0;
  __syncthreads();
  // f(j, i, run) for this thread's entries i = i0 + j < ne
  auto for_entries = [&](auto&& f) {
    u32 q = q0;  // runs started up to entry i0 + j
#pragma unroll
    for (int j = 0; j < EPT; ++j) {
      const u32 i = i0 + (u32)j;
      if (heads & (1u << j)) ++q;
      if (i < ne) f(j, i, q - 1u);  // entry i lies in the last run that starts at or before it
    }
  };
  if (WT) {
    // weighted: every far entry is staged on the compact cursor (its runs add no own-label
    // count); the few of the row's own label are counted and weighed by the group pass.
    // Each run's length is set by the thread that claims it.
    for (u32 r = tid; r < nruns; r += BT_THREADS) s_cnt[r] = s_rf[r + 1] - s_rf[r];
    claim_runs_compact<LT>(nruns, s_rf, s_rb, s_cnt, s_rb, start, D, reinterpret_cast<unsigned long long*>(cursor), ctl);
    __syncthreads();
    for_entries([&](int j, u32 i, u32 run) {
      const u32 base = s_rb[run];
      if (base != SENT) {
        CB[base + (i - s_rf[run])] = x[j];
        CW[base + (i - s_rf[run])] = wt[j];
      }
    });
  } else {
    for_entries([&](int j, u32, u32 run) {
      if ((u32)x[j] != lab[j]) atomicAdd(&s_cnt[run], 1u);
    });
    __syncthreads();
    // s_rb: the run's label, replaced by the place of its first staged entry
    claim_runs_compact<LT>(nruns, s_rf, s_rb, s_cnt, s_rb, start, D, reinterpret_cast<unsigned long long*>(cursor), ctl);
    __syncthreads();
    for_entries([&](int j, u32, u32 run) {
      const u32 base = s_rb[run];
      if ((u32)x[j] != lab[j] && base != SENT) CB[base + atomicAdd(&s_cnt[run], 1u)] = x[j];
    });
  }
}

// One launch for both kinds of tile.  Groups of 8 consecutive workgroups (one per XCD,
// so workgroup i serves block i % 8): the own-span groups first (they carry most
// entries), then the far groups.
template <class LT, bool WT>
__global__ __launch_bounds__(BT_THREADS) void k_gather_blocked(int n, int span, const u32* __restrict__ RPB,
                                                               const int32_t* __restrict__ colb,
                                                               const int32_t* __restrict__ rowb, FarTable ft,
                                                               u32 own_groups, u32 far_groups,
                                                               const LT* __restrict__ labx, const u32* __restrict__ start,
                                                               const u32* __restrict__ D, u32* __restrict__ cursor,
                                                               Ctl* __restrict__ ctl, LT* __restrict__ CB,
                                                               const float* __restrict__ wb, float* __restrict__ CW,
                                                               unsigned long long* __restrict__ IWacc) {
  __shared__ __align__(16) u32 lds[GatherLds<LT, WT>::WORDS];
  __shared__ u32 s_w[BT_THREADS / 64];
  if (ctl->mode == STAGE_ROWS) return;  // this call stages through the row-major copy (k_colscan_rows)
  const u32 y = blockIdx.x % 8u, gi = blockIdx.x / 8u;
  if (y >= (u32)COL_BLOCKS || gi >= own_groups + far_groups) return;
  if (gi < own_groups)
    gather_own_tile<LT, WT>(y, gi, n, span, RPB, colb, labx, start, D, cursor, ctl, CB, wb, CW, IWacc, lds, s_w);
  else
    gather_far_tile<LT, WT>(y, gi - own_groups, ft, colb, rowb, labx, start, D, cursor, ctl, CB, wb, CW, lds, s_w);
}

// Comparison: the segment of ground-truth community a_u receives b_u.
template <bool PRIV, class LT>
__global__ __launch_bounds__(256) void k_cmp_scatter(int n, const int32_t* __restrict__ la, const int32_t* __restrict__ lb,
                                                     int La, int Lb, int chunk, const u32* __restrict__ PM,
                                                     const u32* __restrict__ start, const u32* __restrict__ loc,
                                                     LT* __restrict__ CB) {
  for (size_t u = (size_t)blockIdx.x * blockDim.x + threadIdx.x; u < (size_t)n; u += (size_t)gridDim.x * blockDim.x) {
    int a = la[u];
    u32 lu = loc[u];
    if ((u32)a >= (u32)La || lu == SENT) continue;
    u32 pos = start[a] + lu;
    if (PRIV) pos += PM[(u / chunk) * (size_t)La + a];
    int b = lb[u];
    CB[pos] = ((u32)b < (u32)Lb) ? (LT)b : LabelT<LT>::SENTINEL;
  }
}

// ---------------------------------------------------------------------------
// Group pass.  Persistent workgroups take groups (communities) from work queues
// (wq_next) in the order produced by k_scan_order.  Each group's segment
// CB[start, start+len) holds label values in [0, Lv) (or SENT); the workgroup counts
// them in LDS and hands every (label, count) with count > 0 to the visitor.
//   direct table : Lv counters, when Lv fits the LDS budget and the group is not tiny
//   hash table   : open addressing (keys, counts), capacity a power of two >= 2*min(len, Lv);
//                  when the capacity would exceed the LDS budget the labels are split
//                  into residue classes mod 2^k and counted one class at a time; a class
//                  that overflows is split again.  Every label is counted in exactly one
//                  class, so visitors see each (label, count) once.
constexpr int GBLOCK = 512;
// Score group pass over label spaces that fit a direct LDS table (the batch's too): more,
// smaller workgroups, so that more communities are counted at once (a community's pass
// is bound by its few dependent round trips, not by its thread count)
constexpr int GBLOCK_DIRECT = 256;
// ... and 128 threads for label spaces of at most SMALL_L_MAX ids, whose tables are short
constexpr int GBLOCK_SMALL = 128;
constexpr u32 SMALL_L_MAX = 4096;
// Score group pass over label spaces beyond the direct table: its 128 KB LDS table holds
// one workgroup per CU, so the workgroup takes every wave the CU can hold
constexpr int GBLOCK_WIDE = 1024;
constexpr int STACK = 96;
constexpr u32 WIDE_FIX = 256;  // wrap corrections a 16-bit table can log per group

__device__ __forceinline__ u32 pow2ceil_u32(u32 x) { return x <= 1 ? 1u : 1u << (32 - __clz(x - 1)); }
__device__ __forceinline__ u32 log2_u32(u32 x) { return 31 - __clz(x); }

// Calls f(label) for every entry of a segment: 16-byte vector loads (8 labels of 16
// bits or 4 of 32 bits), two loads in flight per thread, scalar head and tail.
template <class LT, int NT = GBLOCK, class F>
__device__ __forceinline__ void for_each_in_segment(const LT* __restrict__ seg, const u32 len, F&& f) {
  constexpr u32 PER = 16u / sizeof(LT);
  u32 head = (u32)(((16u - ((uintptr_t)seg & 15u)) & 15u) / sizeof(LT));
  if (head > len) head = len;
  const u32 nvec = (len - head) / PER;
  for (u32 e = threadIdx.x; e < head; e += NT) f((u32)seg[e]);
  const uint4* vec = reinterpret_cast<const uint4*>(seg + head);
  auto unpack = [&](const uint4 q) {
    const u32 w4[4] = {q.x, q.y, q.z, q.w};
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      if (sizeof(LT) == 2) {
        f(w4[k] & 0xFFFFu);
        f(w4[k] >> 16);
      } else {
        f(w4[k]);
      }
    }
  };
  u32 i = threadIdx.x;
  for (; i + NT < nvec; i += 2 * NT) {
    const uint4 q0 = vec[i];
    const uint4 q1 = vec[i + NT];
    unpack(q0);
    unpack(q1);
  }
  for (; i < nvec; i += NT) unpack(vec[i]);
  for (u32 e = head + nvec * PER + threadIdx.x; e < len; e += NT) f((u32)seg[e]);
}

// Counts one group's segment CB[base, base+len) (values in [0, Lv) or the sentinel)
// in LDS and hands every (label, count) with count > 0 to the visitor.  hot0 entries of
// the hot label were counted elsewhere (compact staging leaves them out of the segment).
template <class V, class LT, int NT = GBLOCK>
__device__ void group_one(const LT* __restrict__ CB, const u32 base, const u32 len, const u32 g, const u32 Lv,
                          const u32 lds_words, V& vis, Ctl* __restrict__ ctl, const u32 hot0 = 0) {
  extern __shared__ __align__(16) u32 tab[];  // read and cleared as uint4
  __shared__ u32 s_over;
  __shared__ u32 s_hot;
  __shared__ u32 s_nfix;
  __shared__ u32 s_fix_lab[WIDE_FIX];
  __shared__ int s_fix_del[WIDE_FIX];
  __shared__ int s_sp;
  __shared__ u32 s_sr[STACK], s_sm[STACK];
  const int tid = threadIdx.x;
  typename V::State st;
  vis.begin(st, g);
  const u32 M = min(len, Lv);
  u32 hcap = pow2ceil_u32(max(64u, 2u * M));
  // direct when the whole table fits; a visitor with costly visits keeps small segments
  // on the (shorter) hash table
  const bool direct = (Lv <= lds_words) && (V::kDirectWhenFits || 2u * hcap > Lv);
  // 16-bit counters, two per LDS word, for label spaces up to twice the LDS budget
  const bool wide = !direct && Lv > lds_words && ((Lv + 7u) >> 3) * 4u <= lds_words && (4u * hcap > Lv);
  bool use_hash = !direct && !wide;
  if (wide) {
    // Every change of a counter word is one atomic add whose returned value shows
    // whether a 16-bit half wrapped: low half (even label) at 0xFFFF + 1, which also
    // carries 1 into the high half; high half (odd label) at 0xFFFF + 1 from either
    // its own increment or that carry.  Each wrap is logged as a correction (+65536
    // to the wrapped label, -1 to the high label for a carry), so the counts are exact.
    const u32 hot = V::kHotIsGroup ? g : (len ? (u32)CB[base] : 0xFFFFFFFFu);
    const u32 nq = (Lv + 7u) >> 3;  // 16-byte words of the 16-bit table
    uint4* tab4 = reinterpret_cast<uint4*>(tab);
    for (u32 q = tid; q < nq; q += NT) tab4[q] = make_uint4(0u, 0u, 0u, 0u);
    if (tid == 0) {
      s_hot = hot0;
      s_nfix = 0;
    }
    __syncthreads();
    u32 mine = 0;
    auto fix = [&](u32 j, int delta) {
      const u32 i = atomicAdd(&s_nfix, 1u);
      if (i < WIDE_FIX) {
        s_fix_lab[i] = j;
        s_fix_del[i] = delta;
      }
    };
    for_each_in_segment<LT, NT>(CB + base, len, [&](u32 j) {
      if (j == hot) {
        ++mine;
        return;
      }
      if (j >= Lv) return;
      if (j & 1u) {
        const u32 old = atomicAdd(&tab[j >> 1], 0x10000u);
        if ((old >> 16) == 0xFFFFu) fix(j, 1);
      } else {
        const u32 old = atomicAdd(&tab[j >> 1], 1u);
        if ((old & 0xFFFFu) == 0xFFFFu) {
          fix(j, 1);
          fix(j + 1u, 0);  // carry into the high half
          if ((old >> 16) == 0xFFFFu) fix(j + 1u, 1);
        }
      }
    });
    if (mine) atomicAdd(&s_hot, mine);
    __syncthreads();
    const u32 nfix = s_nfix;
    if (nfix > WIDE_FIX) {
      use_hash = true;  // correction log full (more than WIDE_FIX wraps): count again with hashing
    } else {
      if (tid == 0 && s_hot && hot < Lv) vis.visit(st, hot, s_hot);
      auto total = [&](u32 j, u32 half) -> u32 {
        u32 t = half;
        for (u32 i = 0; i < nfix; ++i)
          if (s_fix_lab[i] == j) t += s_fix_del[i] ? 65536u : (u32)-1;
        return t;
      };
      for (u32 q = tid; q < nq; q += NT) {
        const uint4 x = tab4[q];
        const u32 w4[4] = {x.x, x.y, x.z, x.w};
#pragma unroll
        for (int k = 0; k < 8; ++k) {
          const u32 j = 8u * q + (u32)k;
          const u32 half = (w4[k >> 1] >> (16 * (k & 1))) & 0xFFFFu;
          const u32 c = nfix ? total(j, half) : half;
          if (c && j < Lv && j != hot) vis.visit(st, j, c);
        }
      }
    }
    __syncthreads();
  }
  if (direct) {
    // One label usually dominates a segment (the community's own label when scoring,
    // the best-matching detected community when comparing).  Its entries are counted
    // in registers: LDS atomics on a single address would serialise.
    const u32 hot = V::kHotIsGroup ? g : (len ? (u32)CB[base] : 0xFFFFFFFFu);
    const u32 nq = (Lv + 3u) >> 2;  // the table is padded to whole 16-byte words
    uint4* tab4 = reinterpret_cast<uint4*>(tab);
    for (u32 q = tid; q < nq; q += NT) tab4[q] = make_uint4(0u, 0u, 0u, 0u);
    if (tid == 0) s_hot = hot0;
    __syncthreads();
    u32 mine = 0;
    for_each_in_segment<LT, NT>(CB + base, len, [&](u32 j) {
      if (j == hot) ++mine;
      else if (j < Lv) atomicAdd(&tab[j], 1u);
    });
    if (mine) atomicAdd(&s_hot, mine);
    __syncthreads();
    if (tid == 0 && s_hot && hot < Lv) vis.visit(st, hot, s_hot);
    if constexpr (V::kSizesAhead) {
      // the sizes |j| of two table words' labels are loaded before their visits, so
      // that the loads overlap; N is read as 16-byte words up to the table's padding
      // (workspace arrays are 16-byte aligned and padded to 256 bytes)
      const uint4* N4 = reinterpret_cast<const uint4*>(vis.N);
      for (u32 q0 = tid; q0 < nq; q0 += 2u * NT) {
        const u32 q1 = q0 + NT;
        const uint4 n0 = N4[q0];
        uint4 n1 = make_uint4(0u, 0u, 0u, 0u);
        if (q1 < nq) n1 = N4[q1];
        auto visit4 = [&](u32 q, const uint4& nv) {
          const uint4 x = tab4[q];
          if (x.x) vis.visit_n(st, 4u * q, x.x, nv.x);
          if (x.y) vis.visit_n(st, 4u * q + 1u, x.y, nv.y);
          if (x.z) vis.visit_n(st, 4u * q + 2u, x.z, nv.z);
          if (x.w) vis.visit_n(st, 4u * q + 3u, x.w, nv.w);
        };
        visit4(q0, n0);
        if (q1 < nq) visit4(q1, n1);
      }
    } else {
      for (u32 q = tid; q < nq; q += NT) {
        const uint4 x = tab4[q];
        if (x.x) vis.visit(st, 4u * q, x.x);
        if (x.y) vis.visit(st, 4u * q + 1u, x.y);
        if (x.z) vis.visit(st, 4u * q + 2u, x.z);
        if (x.w) vis.visit(st, 4u * q + 3u, x.w);
      }
    }
  }
  if (use_hash) {
    // The segment's dominant label is counted in registers during the first pass and
    // never enters the table.  When the table must be split, the first split gives each
    // residue class about 2*capmax of the M entries, assuming at most M/2 distinct keys
    // (repeated and dominant labels keep them below that); a class that still
    // overflows is split again.
    const u32 hot = V::kHotIsGroup ? g : (len ? (u32)CB[base] : 0xFFFFFFFFu);
    const u32 capmax = 1u << log2_u32(lds_words / 2u);
    u32 classes = 1;
    if (hcap > capmax) {
      classes = pow2ceil_u32((M + 2u * capmax - 1u) / (2u * capmax));
      if (classes > 32u) classes = 32u;
      hcap = capmax;
    }
    const u32 lg = log2_u32(hcap);
    u32* keys = tab;
    u32* cnt = tab + hcap;
    if (tid == 0) {
      s_sp = 0;
      s_hot = hot0;
      for (int r = (int)classes - 1; r >= 0; --r) { s_sr[s_sp] = (u32)r; s_sm[s_sp] = classes; ++s_sp; }
    }
    __syncthreads();
    u32 mine = 0;
    bool first = true;
    for (;;) {
      const int sp = s_sp;
      if (sp == 0) break;
      const u32 r = s_sr[sp - 1], mod = s_sm[sp - 1];
      __syncthreads();
      if (tid == 0) { s_sp = sp - 1; s_over = 0; }
      for (u32 s = tid; s < hcap; s += NT) { keys[s] = EMPTY; cnt[s] = 0; }
      __syncthreads();
      bool over = false;
      for_each_in_segment<LT, NT>(CB + base, len, [&](u32 j) {
        if (j == hot) {
          if (first) ++mine;
          return;
        }
        if (j >= Lv || (j & (mod - 1u)) != r) return;
        u32 h = hash_slot(j, lg);
        for (u32 p = 0; p < hcap; ++p) {
          const u32 k = keys[h];
          if (k == EMPTY) {
            const u32 old = atomicCAS(&keys[h], EMPTY, j);
            if (old == EMPTY || old == j) {
              atomicAdd(&cnt[h], 1u);
              return;
            }
          } else if (k == j) {
            atomicAdd(&cnt[h], 1u);
            return;
          }
          h = (h + 1u) & (hcap - 1u);
        }
        over = true;
      });
      if (over) s_over = 1;
      first = false;
      __syncthreads();
      if (s_over) {
        if (tid == 0) {
          if (s_sp + 2 <= STACK && mod < 0x80000000u) {
            s_sr[s_sp] = r + mod; s_sm[s_sp] = 2u * mod; ++s_sp;
            s_sr[s_sp] = r; s_sm[s_sp] = 2u * mod; ++s_sp;
          } else {
            atomicOr(&ctl->flags, F_STACK);
          }
        }
        __syncthreads();
        continue;
      }
      for (u32 s = tid; s < hcap; s += NT) {
        u32 k = keys[s];
        if (k != EMPTY) {
          vis.visit(st, k, cnt[s]);
          vis.settle(st);  // slots hold labels in an order the atomics chose
        }
      }
      __syncthreads();
    }
    if (mine) atomicAdd(&s_hot, mine);
    __syncthreads();
    if (tid == 0 && s_hot && hot < Lv) {
      vis.visit(st, hot, s_hot);
      vis.settle(st);
    }
  }
  vis.settle(st);  // direct and 16-bit tables: each thread met its labels in a fixed order
  vis.finish(st, g);
  __syncthreads();
}

template <class V, class LT, int NT = GBLOCK>
// cur64 (compact staging, else null): low word = segment length, high word = entries of
// the group's own label left out of the segment; otherwise seg_len gives the length.
// NT threads per workgroup.
__global__ __launch_bounds__(NT) void k_groups(const LT* __restrict__ CB, const u32* __restrict__ seg_start,
                                                   const u32* __restrict__ seg_len, const u32* __restrict__ order,
                                                   Ctl* __restrict__ ctl, u32 Lv, u32 lds_words, V vis,
                                                   const unsigned long long* __restrict__ cur64, u32* __restrict__ wq,
                                                   bool big_only = false) {
  __shared__ u32 s_item;
  const u32 K = big_only ? ctl->kbig : ctl->K;  // big_only: the small groups go to k_groups_wave
  const bool compact = cur64 && ctl->mode != STAGE_ROWS;
  u32 q = blockIdx.x % WQ_QUEUES, left = WQ_QUEUES;  // thread 0's queue state
  for (;;) {
    if (threadIdx.x == 0) s_item = wq_next(wq, K, q, left);
    __syncthreads();
    const u32 item = s_item;
    __syncthreads();
    if (item >= K) break;
    const u32 g = order[item];
    const unsigned long long c = compact ? cur64[g] : (unsigned long long)seg_len[g];
    group_one<V, LT, NT>(CB, seg_start[g], (u32)c, g, Lv, lds_words, vis, ctl, (u32)(c >> 32));
  }
}

// Group pass, one wave per group, for the groups after ctl->kbig in the order (segments
// of fewer than GW_SPLIT entries; 16-bit labels).  A workgroup-wide pass spends most of
// such a small group waiting on its barriers and its few dependent loads; here every
// wave of a CU works on a group of its own, with no barrier at all.  Each wave counts its
// segment in its own LDS hash table of 32-bit words (label << 16 | count): the labels are
// below 65535 (0xFFFF marks an empty slot, never a label) and a count is at most the
// segment length, below 2^16.  Fewer distinct labels than slots (GW_SLOTS > GW_SPLIT - 1)
// means every probe sequence ends.  The dominant label is counted in registers as in
// group_one.  V provides finish_wave (the visitor's reduction over one wave).
constexpr int GW_WAVES = 8;
constexpr u32 GW_SLOTS = 2048;
constexpr int GW_WORDS_PER_LANE = 5;  // 320 16-byte words cover GW_SPLIT - 1 entries at any alignment
static_assert(64 * GW_WORDS_PER_LANE * 8 >= (int)GW_SPLIT - 1 + 7 + 8, "wave segment words");
static_assert(GW_SLOTS % (64 * 8) == 0, "visit batches");
static_assert(GW_SLOTS > GW_SPLIT - 1, "a wave's table must have an empty slot for every segment it takes");
// One group counted by the calling wave in its table `tab` (GW_SLOTS words): segment
// CB[base, base + len) with len < GW_SPLIT, hot0 entries of the hot label left out of it
// (compact staging).  Every term the visitor gets is settled on its own (slot order follows
// the atomics), so a group's result does not depend on which lanes met which labels.
template <class V>
__device__ __forceinline__ void wave_group_one(u32* tab, const uint16_t* __restrict__ CB, u32 base, u32 len, u32 hot0, u32 g,
                                               u32 Lv, V& vis, Ctl* __restrict__ ctl) {
  const u32 lane = threadIdx.x & 63u;
  for (u32 i = lane; i < GW_SLOTS; i += 64) tab[i] = EMPTY;
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");  // the wave's clears land before its inserts
  // The segment's 16-byte words, all loaded before the first is used: word w of the
  // aligned range holds entries a0 + 8w .. a0 + 8w + 7 (entries outside the segment are
  // skipped; the word past its end still lies inside the workspace's carved array).
  const u32 a0 = base & ~7u;
  const u32 nw = (base + len - a0 + 7u) >> 3;  // at most GW_WORDS_PER_LANE * 64 words
  const uint4* cb4 = reinterpret_cast<const uint4*>(CB + a0);
  uint4 wv[GW_WORDS_PER_LANE];
#pragma unroll
  for (int i = 0; i < GW_WORDS_PER_LANE; ++i) {
    const u32 wi = lane + 64u * (u32)i;
    wv[i] = wi < nw ? cb4[wi] : make_uint4(0xFFFFFFFFu, 0xFFFFFFFFu, 0xFFFFFFFFu, 0xFFFFFFFFu);
  }
  const u32 hot = V::kHotIsGroup ? g : (len ? (u32)CB[base] : 0xFFFFFFFFu);
  u32 mine = 0, lost = 0;
#pragma unroll
  for (int i = 0; i < GW_WORDS_PER_LANE; ++i) {
    const u32 w4[4] = {wv[i].x, wv[i].y, wv[i].z, wv[i].w};
    const u32 e0 = a0 + 8u * (lane + 64u * (u32)i);
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const u32 e = e0 + (u32)k;
      const u32 j = (w4[k >> 1] >> (16 * (k & 1))) & 0xFFFFu;
      if (e < base || e >= base + len) continue;
      if (j == hot) {
        ++mine;
        continue;
      }
      if (j >= Lv) continue;
      u32 h = hash_slot(j, 11);  // log2(GW_SLOTS)
      bool done = false;
      for (u32 p = 0; p < GW_SLOTS && !done; ++p) {
        const u32 t = tab[h];
        if ((t >> 16) == j) {
          atomicAdd(&tab[h], 1u);
          done = true;
        } else if (t == EMPTY) {
          const u32 old = atomicCAS(&tab[h], EMPTY, (j << 16) | 1u);
          if (old == EMPTY) {
            done = true;
          } else if ((old >> 16) == j) {
            atomicAdd(&tab[h], 1u);
            done = true;
          }
        }
        if (!done) h = (h + 1u) & (GW_SLOTS - 1u);
      }
      lost += done ? 0u : 1u;  // never expected (the table always has an empty slot)
    }
  }
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");  // every insert lands before the reads
  if (lost) atomicOr(&ctl->flags, F_STACK);
  typename V::State st;
  vis.begin_wave(st, g);
  // the lane's slots in batches of 8: the batch's sizes are loaded before its visits
  for (u32 i0 = lane; i0 < GW_SLOTS; i0 += 64u * 8u) {
    u32 k[8], sz[8];
#pragma unroll
    for (int b = 0; b < 8; ++b) k[b] = tab[i0 + 64u * (u32)b];
#pragma unroll
    for (int b = 0; b < 8; ++b) sz[b] = k[b] != EMPTY ? vis.size_of(k[b] >> 16) : 0u;
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      if (k[b] != EMPTY) {
        vis.visit_n(st, k[b] >> 16, k[b] & 0xFFFFu, sz[b]);
        vis.settle(st);
      }
    }
  }
  const u32 nhot = (u32)wave_sum_u64(mine) + hot0;
  if (lane == 0 && nhot && hot < Lv) {
    vis.visit(st, hot, nhot);
    vis.settle(st);
  }
  vis.finish_wave(st, g);
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");  // the table's reads end before the next clears
}

// cur64 (compact staging of a column-blocked graph, else null): as in k_groups.
template <class V>
__global__ __launch_bounds__(64 * GW_WAVES) void k_groups_wave(const uint16_t* __restrict__ CB, const u32* __restrict__ seg_start,
                                                              const u32* __restrict__ seg_len, const u32* __restrict__ order,
                                                              Ctl* __restrict__ ctl, u32 Lv, V vis, u32* __restrict__ wq,
                                                              const unsigned long long* __restrict__ cur64 = nullptr) {
  __shared__ u32 s_tab[GW_WAVES * GW_SLOTS];
  const u32 lane = threadIdx.x & 63u, w = threadIdx.x >> 6;
  u32* tab = s_tab + w * GW_SLOTS;
  const u32 k0 = ctl->kbig, K = ctl->K;
  const u32 nsmall = K > k0 ? K - k0 : 0u;
  const bool compact = cur64 && ctl->mode != STAGE_ROWS;
  u32 q = (blockIdx.x * GW_WAVES + w) % WQ_QUEUES, left = WQ_QUEUES;  // lane 0's queue state
  for (;;) {
    u32 item = 0;
    if (lane == 0) item = wq_next(wq + WQ_WAVE, nsmall, q, left);
    item = __shfl(item, 0, 64);
    if (item == 0xFFFFFFFFu) break;
    const u32 g = order[k0 + item];
    const unsigned long long c = compact ? cur64[g] : (unsigned long long)seg_len[g];
    wave_group_one<V>(tab, CB, seg_start[g], min((u32)c, GW_SPLIT - 1u), (u32)(c >> 32), g, Lv, vis, ctl);
  }
}

// block reduction helpers for the visitors (GBLOCK threads)
__device__ __forceinline__ u128 block_sum_u128(u128 x, u64* sh_lo, u64* sh_hi) {
  x = wave_sum_u128(x);
  int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) { sh_lo[w] = (u64)x; sh_hi[w] = (u64)(x >> 64); }
  __syncthreads();
  u128 r = 0;
  if (threadIdx.x == 0)
    for (int i = 0; i < (int)(blockDim.x >> 6); ++i) r += ((u128)sh_hi[i] << 64) | sh_lo[i];
  __syncthreads();
  return r;
}
__device__ __forceinline__ u64 block_sum_u64(u64 x, u64* sh) {
  x = wave_sum_u64(x);
  int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) sh[w] = x;
  __syncthreads();
  u64 r = 0;
  if (threadIdx.x == 0)
    for (int i = 0; i < (int)(blockDim.x >> 6); ++i) r += sh[i];
  __syncthreads();
  return r;
}
// Score visitor: for community g, label j with count x in g's segment:
//   j == g  ->  x = 2|E_g^in|
//   j != g  ->  x = |E_{g,j}|; contributes |E_gj|/(2|E|) * |E_gj|/(|g||j|) to g's
//               split-penalty sum (Eq. 9); pairs with j > g are counted (and exported).
struct ScoreVis {
  static constexpr bool kHotIsGroup = true;
  static constexpr bool kDirectWhenFits = true;
  static constexpr bool kSizesAhead = true;  // visit_n: N (L entries, padded to 16 bytes) read as 16-byte words
  const u32* N;
  double twom;
  u32* I;
  u32* NP;
  u64* PEN;
  int32_t* eci;
  int32_t* ecj;
  int64_t* ecnt;
  long long ecap;
  Ctl* ctl;
  struct State {
    Frac96Sum pen;
    double acc;  // terms not yet in pen
    u32 np;
    u32 g;
    double denom;
  };
  __device__ void begin(State& st, u32 g) {
    st.pen = Frac96Sum();
    st.acc = 0.0;
    st.np = 0;
    st.g = g;
    st.denom = twom * (double)N[g];
    if (threadIdx.x == 0) I[g] = 0;  // overwritten by the thread that meets label g
  }
  // k_groups_wave: lane 0 of the group's wave clears I[g]
  __device__ void begin_wave(State& st, u32 g) {
    st.pen = Frac96Sum();
    st.acc = 0.0;
    st.np = 0;
    st.g = g;
    st.denom = twom * (double)N[g];
    if ((threadIdx.x & 63) == 0) I[g] = 0;
  }
  __device__ u32 size_of(u32 j) const { return N[j]; }
  __device__ void visit(State& st, u32 j, u32 x) { visit_n(st, j, x, N[j]); }
  // the same with |j| = nj already loaded
  __device__ void visit_n(State& st, u32 j, u32 x, u32 nj) {
    if (j == st.g) {
      I[j] = x;
      return;
    }
    const double xd = (double)x;
    st.acc += xd * xd * recip_nr(st.denom * (double)nj);  // a term <= x / 2m <= 1/2
    if (j > st.g) {
      st.np += 1;
      if (ecap > 0) {
        unsigned long long idx = atomicAdd(&ctl->export_count, 1ull);
        if ((long long)idx < ecap) { eci[idx] = (int32_t)st.g; ecj[idx] = (int32_t)j; ecnt[idx] = (int64_t)x; }
      }
    }
  }
  // Moves the thread's pending terms into the exact sum.  The group pass settles once per
  // group where a thread visits its labels in a fixed order (the same binary64 sum on
  // every run), and after each visit where the order varies, so results never depend on
  // the order of atomics.
  __device__ void settle(State& st) {
    if (st.acc != 0.0) st.pen.add_wide(st.acc);  // at most 1/2 per visit
    st.acc = 0.0;
  }
  // Reduces the threads' sums with one barrier (waves first, then the waves in order);
  // the caller's next barrier protects the LDS partials.
  __device__ void finish(State& st, u32 g) {
    __shared__ u64 r_lo[GBLOCK_WIDE / 64], r_hi[GBLOCK_WIDE / 64], r_np[GBLOCK_WIDE / 64];  // up to 16 waves
    const u128 pen = wave_sum_u128(st.pen.value());
    const u64 np = wave_sum_u64(st.np);
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
      r_lo[w] = (u64)pen;
      r_hi[w] = (u64)(pen >> 64);
      r_np[w] = np;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      u128 p = 0;
      u64 q = 0;
      for (int i = 0; i < (int)(blockDim.x >> 6); ++i) {
        p += ((u128)r_hi[i] << 64) | r_lo[i];
        q += r_np[i];
      }
      PEN[2 * (size_t)g] = (u64)p;
      PEN[2 * (size_t)g + 1] = (u64)(p >> 64);
      NP[g] = (u32)q;
    }
  }
  // The same over one wave (k_groups_wave): no barrier, lane 0 writes.
  __device__ void finish_wave(State& st, u32 g) {
    const u128 pen = wave_sum_u128(st.pen.value());
    const u64 np = wave_sum_u64(st.np);
    if ((threadIdx.x & 63) == 0) {
      PEN[2 * (size_t)g] = (u64)pen;
      PEN[2 * (size_t)g + 1] = (u64)(pen >> 64);
      NP[g] = (u32)np;
    }
  }
};

// ---------------------------------------------------------------------------
// Weighted group pass (edge-weighted graphs; labels fit a direct LDS table).  Per
// community g, besides everything ScoreVis computes from the counts:
//   SW[g] = sum of the weights in g's segment = strength sum s(g)       (x 2^55, exact)
//   IW[g] = sum of the weights of entries labelled g = 2 w_in(g)         (x 2^55, exact)
//   PENW[g] = sum_{j != g} w(g,j) d_{g,j} / (2W), d_{g,j} = |E_gj| / (|g||j|)   (x 2^96)
// The first pass counts labels exactly as the unweighted pass does.  The second pass,
// once the table holds every count |E_gj|, reads labels and weights together: entry
// (j, w) adds w to the weight sums and, for j != g, w |E_gj| / (2W |g| |j|) to the
// penalty, truncated to a multiple of 2^-96 (term by term, so the sum is exact).  With
// compact staging (column-blocked graphs) the segment holds only entries of other
// labels (and far entries): the edge pass has already counted the own-label entries
// (high word of the cursor) and summed their weights into IW[g], which both sums add.
struct WeightedOut {
  u64* SW;
  u64* IW;
  u64* PENW;
  const double* invN;  // 1/|j| per label (0 for empty labels)
  double twoW;
};



// Calls f(label, weight) for every entry of a segment of labels and weights (both arrays
// 16-byte aligned at index 0): 4 entries per load once the index is a multiple of 4.
// One load in flight per thread: the weighted pass is register-bound, and more waves
// hide the latency better than a second load would.
template <class LT, class F>
__device__ __forceinline__ void for_each_weighted(const LT* __restrict__ lab, const float* __restrict__ wt, const u32 base,
                                                  const u32 len, F&& f) {
  u32 head = (4u - (base & 3u)) & 3u;
  if (head > len) head = len;
  const u32 nvec = (len - head) / 4u;
  for (u32 e = threadIdx.x; e < head; e += GBLOCK) f((u32)lab[base + e], wt[base + e]);
  const u32 b4 = base + head;  // a multiple of 4
  const float4* wv = reinterpret_cast<const float4*>(wt + b4);
  auto labels4 = [&](u32 i, u32 (&j)[4]) {
    if (sizeof(LT) == 2) {
      const uint2 q = reinterpret_cast<const uint2*>(lab + b4)[i];
      j[0] = q.x & 0xFFFFu; j[1] = q.x >> 16; j[2] = q.y & 0xFFFFu; j[3] = q.y >> 16;
    } else {
      const uint4 q = reinterpret_cast<const uint4*>(lab + b4)[i];
      j[0] = q.x; j[1] = q.y; j[2] = q.z; j[3] = q.w;
    }
  };
  for (u32 i = threadIdx.x; i < nvec; i += GBLOCK) {
    u32 j0[4];
    labels4(i, j0);
    const float4 w0 = wv[i];
    f(j0[0], w0.x); f(j0[1], w0.y); f(j0[2], w0.z); f(j0[3], w0.w);
  }
  for (u32 e = head + nvec * 4u + threadIdx.x; e < len; e += GBLOCK) f((u32)lab[base + e], wt[base + e]);
}

template <class LT>
__device__ void group_one_w(const LT* __restrict__ CB, const float* __restrict__ CW, const u32 base, const u32 len,
                            const u32 g, const u32 Lv, ScoreVis& vis, const WeightedOut& wo, const u32 hot0,
                            const bool own_in_iw) {
  extern __shared__ __align__(16) u32 tab[];  // read and cleared as uint4
  __shared__ u32 s_hot;
  __shared__ u64 r_w[6][GBLOCK / 64];
  const int tid = threadIdx.x;
  ScoreVis::State st;
  vis.begin(st, g);
  const u32 nq = (Lv + 3u) >> 2;
  uint4* tab4 = reinterpret_cast<uint4*>(tab);
  for (u32 q = tid; q < nq; q += GBLOCK) tab4[q] = make_uint4(0u, 0u, 0u, 0u);
  if (tid == 0) s_hot = hot0;
  __syncthreads();
  u32 mine = 0;
  for_each_in_segment<LT>(CB + base, len, [&](u32 j) {
    if (j == g) ++mine;
    else if (j < Lv) atomicAdd(&tab[j], 1u);
  });
  if (mine) atomicAdd(&s_hot, mine);
  __syncthreads();
  if (tid == 0 && s_hot && g < Lv) vis.visit(st, g, s_hot);
  for (u32 q = tid; q < nq; q += GBLOCK) {
    const uint4 x = tab4[q];
    if (x.x) vis.visit(st, 4u * q, x.x);
    if (x.y) vis.visit(st, 4u * q + 1u, x.y);
    if (x.z) vis.visit(st, 4u * q + 2u, x.z);
    if (x.w) vis.visit(st, 4u * q + 3u, x.w);
  }
  // second pass: weight sums and the weighted split penalty, every count now in the table.
  // Branch-free: an entry of label g adds 0 to the penalty, a label outside [0, Lv) (only
  // with a label error, which voids the result) reads slot g instead.
  vis.settle(st);  // the table gave each thread its labels in a fixed order
  WeightSum sall, shot;
  Frac96Sum pw;
  const double kg = 1.0 / (wo.twoW * (double)vis.N[g]);
  for_each_weighted<LT>(CB, CW, base, len, [&](u32 j, float w) {
    u64 vlo, vhi;
    WeightSum::split(w, vlo, vhi);
    sall.add(vlo, vhi);
    const bool own = j == g;
    shot.add(own ? vlo : 0ull, own ? vhi : 0ull);
    const u32 jj = j < Lv ? j : g;
    const double f = own ? 0.0 : (double)tab[jj] * wo.invN[jj];
    pw.add((double)w * f * kg);
  });
  vis.finish(st, g);  // one barrier; the reads of tab above are done before anyone clears it
  {
    const u128 a = wave_sum_u128(sall.value()), b = wave_sum_u128(shot.value()), c = wave_sum_u128(pw.value());
    const int w = tid >> 6;
    if ((tid & 63) == 0) {
      r_w[0][w] = (u64)a;
      r_w[1][w] = (u64)(a >> 64);
      r_w[2][w] = (u64)b;
      r_w[3][w] = (u64)(b >> 64);
      r_w[4][w] = (u64)c;
      r_w[5][w] = (u64)(c >> 64);
    }
  }
  __syncthreads();
  if (tid == 0) {
    // own-label weights the edge pass summed into IW (compact staging)
    const u128 iw0 = own_in_iw ? ((u128)wo.IW[2 * (size_t)g + 1] << 64) | wo.IW[2 * (size_t)g] : (u128)0;
    u128 a = iw0, b = iw0, c = 0;
    for (int i = 0; i < GBLOCK / 64; ++i) {
      a += ((u128)r_w[1][i] << 64) | r_w[0][i];
      b += ((u128)r_w[3][i] << 64) | r_w[2][i];
      c += ((u128)r_w[5][i] << 64) | r_w[4][i];
    }
    wo.SW[2 * (size_t)g] = (u64)a;
    wo.SW[2 * (size_t)g + 1] = (u64)(a >> 64);
    wo.IW[2 * (size_t)g] = (u64)b;
    wo.IW[2 * (size_t)g + 1] = (u64)(b >> 64);
    wo.PENW[2 * (size_t)g] = (u64)c;
    wo.PENW[2 * (size_t)g + 1] = (u64)(c >> 64);
  }
  __syncthreads();
}

template <class LT>
__global__ __launch_bounds__(GBLOCK, 6) void k_groups_w(const LT* __restrict__ CB, const float* __restrict__ CW,
                                                     const u32* __restrict__ seg_start, const u32* __restrict__ seg_len,
                                                     const u32* __restrict__ order, Ctl* __restrict__ ctl, u32 Lv,
                                                     ScoreVis vis, WeightedOut wo,
                                                     const unsigned long long* __restrict__ cur64, u32* __restrict__ wq) {
  __shared__ u32 s_item;
  const u32 K = ctl->K;
  u32 q = blockIdx.x % WQ_QUEUES, left = WQ_QUEUES;  // thread 0's queue state (see wq_next)
  for (;;) {
    if (threadIdx.x == 0) s_item = wq_next(wq, K, q, left);
    __syncthreads();
    const u32 item = s_item;
    __syncthreads();
    if (item >= K) break;
    const u32 g = order[item];
    u32 len = seg_len[g], hot0 = 0;
    if (cur64) {  // compact staging: length and own-label count in the cursor, own-label weights in IW
      const unsigned long long c = cur64[g];
      len = (u32)c;
      hot0 = (u32)(c >> 32);
    }
    group_one_w<LT>(CB, CW, seg_start[g], len, g, Lv, vis, wo, hot0, cur64 != nullptr);
  }
}

// 1/|j| for every label id (0 where no node carries it), for the weighted penalty.
__global__ void k_inv_sizes(int L, const u32* __restrict__ N, double* __restrict__ invN) {
  for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < L; c += gridDim.x * blockDim.x)
    invN[c] = N[c] ? 1.0 / (double)N[c] : 0.0;
}

// Comparison visitor: row i of the contingency table, column j, cell x = |c_i ∩ c'_j|.
// The information terms need one logarithm per cell: with N = sum of the cells, the
// rows summing to a_i and the columns to b_j,
//   sum (x/N) log(x N / (a_i b_j)) = S + log N - S_a - S_b          (Eq. 2 numerator)
//   sum (x/N) log(x^2 / (a_i b_j)) = 2 S - S_a - S_b                 (Eq. 1, negated)
// where S = sum over cells of (x/N) log x, S_a = sum_i (a_i/N) log a_i, S_b likewise.
// RXL[i] receives row i's part of S (fix96); S_a and S_b are summed in the final pass.
struct CmpVis {
  static constexpr bool kHotIsGroup = false;
  static constexpr bool kDirectWhenFits = false;
  static constexpr bool kSizesAhead = false;
  const u32* A;   // |c_i|
  const u32* B;   // |c'_j|
  double Nd;
  u32* COLMAX;
  u64* RA11;
  u32* RMAX;
  double* RF;
  u64* RXL;
  int32_t* eci;
  int32_t* ecj;
  int64_t* ecnt;
  long long ecap;
  Ctl* ctl;
  u32* wq;  // non-zero cells are counted per work queue (wq_sum): one address would serialise
  struct State {
    u64 a11;
    u32 rmax;
    double fmax;
    Frac96Sum xl;  // S in fixed point; each term lies in [0, log N]
    u32 g;
    u32 ai;
    u32 nz;
  };
  __device__ void begin(State& st, u32 g) {
    st.a11 = 0;
    st.rmax = 0;
    st.fmax = 0.0;
    st.xl = Frac96Sum();
    st.g = g;
    st.ai = A[g];
    st.nz = 0;
  }
  __device__ void settle(State&) {}  // every visit adds exactly
  __device__ void begin_wave(State& st, u32 g) { begin(st, g); }
  __device__ u32 size_of(u32 j) const { return B[j]; }
  __device__ void visit(State& st, u32 j, u32 x) { visit_n(st, j, x, B[j]); }
  // the same with |c'_j| = bj already loaded
  __device__ void visit_n(State& st, u32 j, u32 x, u32 bj) {
    st.a11 += (u64)x * (u64)(x - 1u) / 2u;
    st.rmax = max(st.rmax, x);
    double f = 2.0 * (double)x / (double)((u64)st.ai + (u64)bj);   // Eq. 3 ratio
    st.fmax = f > st.fmax ? f : st.fmax;
    st.xl.add_wide((double)x / Nd * log((double)x));  // the cell's part of S, truncated to 2^-96 as fix96 does
    atomicMax(&COLMAX[j], x);
    st.nz += 1;
    if (ecap > 0) {
      unsigned long long idx = atomicAdd(&ctl->export_count, 1ull);
      if ((long long)idx < ecap) { eci[idx] = (int32_t)st.g; ecj[idx] = (int32_t)j; ecnt[idx] = (int64_t)x; }
    }
  }
  // One barrier for all six reductions (see ScoreVis::finish).
  __device__ void finish(State& st, u32 g) {
    constexpr int NW = GBLOCK / 64;
    __shared__ u64 r_mlo[NW], r_mhi[NW], r_a11[NW], r_nz[NW];
    __shared__ u32 r_max[NW];
    __shared__ double r_f[NW];
    {
      const u128 wm = wave_sum_u128(st.xl.value());
      const u64 wa = wave_sum_u64(st.a11), wn = wave_sum_u64(st.nz);
      const u32 wx = wave_max_u32(st.rmax);
      const double wf = wave_max_f64(st.fmax);
      const int w = threadIdx.x >> 6;
      if ((threadIdx.x & 63) == 0) {
        r_mlo[w] = (u64)wm;
        r_mhi[w] = (u64)(wm >> 64);
        r_a11[w] = wa;
        r_nz[w] = wn;
        r_max[w] = wx;
        r_f[w] = wf;
      }
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      u128 xl = 0;
      u64 a11 = 0, nz = 0;
      u32 rmax = 0;
      double fmax = 0.0;
      for (int i = 0; i < (int)(blockDim.x >> 6); ++i) {
        xl += ((u128)r_mhi[i] << 64) | r_mlo[i];
        a11 += r_a11[i];
        nz += r_nz[i];
        rmax = max(rmax, r_max[i]);
        fmax = r_f[i] > fmax ? r_f[i] : fmax;
      }
      atomicAdd(wq_sum(wq, blockIdx.x % WQ_QUEUES), (unsigned long long)nz);
      RA11[g] = a11;
      RMAX[g] = rmax;
      RF[g] = fmax;
      RXL[2 * (size_t)g] = (u64)xl;
      RXL[2 * (size_t)g + 1] = (u64)(xl >> 64);
    }
  }
  // The same reductions over one wave (k_groups_wave): no barrier, lane 0 writes.
  __device__ void finish_wave(State& st, u32 g) {
    const u128 xl = wave_sum_u128(st.xl.value());
    const u64 a11 = wave_sum_u64(st.a11), nz = wave_sum_u64(st.nz);
    const u32 rmax = wave_max_u32(st.rmax);
    const double fmax = wave_max_f64(st.fmax);
    if ((threadIdx.x & 63) == 0) {
      atomicAdd(wq_sum(wq, blockIdx.x % WQ_QUEUES), (unsigned long long)nz);
      RA11[g] = a11;
      RMAX[g] = rmax;
      RF[g] = fmax;
      RXL[2 * (size_t)g] = (u64)xl;
      RXL[2 * (size_t)g + 1] = (u64)(xl >> 64);
    }
  }
};

// ---------------------------------------------------------------------------
// Final reductions.  Stage 1: block b reduces a fixed contiguous range of labels
// (thread t takes every blockDim-th label of it), then combines its threads in a
// fixed order.  Stage 2: one block combines the stage-1 partials in block order.
// Integer and fixed-point sums are exact; double sums have a fixed order, so the
// result is bitwise reproducible.
constexpr int FBLOCK = 256;

// Block sums of NU u64, NX u128 and NF binary64 fields of an FBLOCK-thread block with one
// barrier: a fixed butterfly in each wave, then thread 0 adds the waves in order, which
// gives each field the value a block sum of that field alone would.  The totals replace
// the inputs in thread 0 only.
template <int NU, int NX, int NF>
__device__ __forceinline__ void block_sum_fields(u64 (&u)[NU], u128 (&x)[NX], double (&f)[NF]) {
  constexpr int NW = FBLOCK / 64;
  __shared__ u64 s_u[NU][NW];
  __shared__ u64 s_x[2 * NX][NW];
  __shared__ double s_f[NF][NW];
#pragma unroll
  for (int k = 0; k < NU; ++k) u[k] = wave_sum_u64(u[k]);
#pragma unroll
  for (int k = 0; k < NX; ++k) x[k] = wave_sum_u128(x[k]);
#pragma unroll
  for (int k = 0; k < NF; ++k)
    for (int o = 32; o > 0; o >>= 1) f[k] += __shfl_xor(f[k], o, 64);
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
#pragma unroll
    for (int k = 0; k < NU; ++k) s_u[k][w] = u[k];
#pragma unroll
    for (int k = 0; k < NX; ++k) {
      s_x[2 * k][w] = (u64)x[k];
      s_x[2 * k + 1][w] = (u64)(x[k] >> 64);
    }
#pragma unroll
    for (int k = 0; k < NF; ++k) s_f[k][w] = f[k];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int k = 0; k < NU; ++k) {
      u[k] = 0;
      for (int i = 0; i < NW; ++i) u[k] += s_u[k][i];
    }
#pragma unroll
    for (int k = 0; k < NX; ++k) {
      x[k] = 0;
      for (int i = 0; i < NW; ++i) x[k] += ((u128)s_x[2 * k + 1][i] << 64) | s_x[2 * k][i];
    }
#pragma unroll
    for (int k = 0; k < NF; ++k) {
      f[k] = 0.0;
      for (int i = 0; i < NW; ++i) f[k] += s_f[k][i];
    }
  }
}

struct ScorePart {
  u64 K, sein, seout, sD2, np, pen_lo, pen_hi, pad;
  double qds_a, s_dens, s_contr, s_exp, s_cond, pad2[3];
};

struct PerComm {
  int64_t* size;
  int64_t* degsum;
  int64_t* ein;
  int64_t* eout;
  double* intra_density;
  double* contraction;
  double* expansion;
  double* conductance;
  double* q_term;
  double* qds_term;
  double* w_in;      // weighted graphs only
  double* strength;  // weighted graphs only
};

__device__ void score_final1_body(int L, const u32* __restrict__ N, const u32* __restrict__ D, const u32* __restrict__ I,
                                  const u32* __restrict__ NP, const u64* __restrict__ PEN, double twom, const PerComm& pc,
                                  ScorePart* __restrict__ parts, int blk, int G) {
  const int R = (L + G - 1) / G;
  const int c0 = blk * R, c1 = min(L, c0 + R);
  const double m = 0.5 * twom;
  u64 K = 0, sein = 0, seout = 0, sD2 = 0, np = 0;
  u128 pen = 0;
  double qds_a = 0, s_dens = 0, s_contr = 0, s_exp = 0, s_cond = 0;
  for (int c = c0 + threadIdx.x; c < c1; c += FBLOCK) {
    const u32 nc = N[c];
    int64_t o_size = 0, o_deg = 0, o_ein = 0, o_eout = 0;
    double o_d = 0, o_contr = 0, o_exp = 0, o_cond = 0, o_q = 0, o_qds = 0;
    if (nc > 0) {
      const u32 Dc = D[c], Ic = I[c];
      const u32 ein = Ic / 2u, eout = Dc - Ic;
      const u128 pc128 = ((u128)PEN[2 * (size_t)c + 1] << 64) | PEN[2 * (size_t)c];
      const double d = nc >= 2 ? (2.0 * (double)ein) / (double)((u64)nc * (u64)(nc - 1u)) : 0.0;
      const double tot = (double)Dc / twom;
      const double tdc = tot * d;
      const double qa = (double)ein / m * d - tdc * tdc;
      const double penc = unfix96(pc128);
      o_size = nc; o_deg = Dc; o_ein = ein; o_eout = eout;
      o_d = d;
      o_contr = 2.0 * (double)ein / (double)nc;
      o_exp = (double)eout / (double)nc;
      o_cond = Dc > 0 ? (double)eout / (double)Dc : 0.0;
      o_q = (double)ein / m - tot * tot;
      o_qds = qa - penc;
      K += 1; sein += ein; seout += eout; sD2 += (u64)Dc * (u64)Dc; np += NP[c]; pen += pc128;
      qds_a += qa; s_dens += o_d; s_contr += o_contr; s_exp += o_exp; s_cond += o_cond;
    }
    if (pc.size) pc.size[c] = o_size;
    if (pc.degsum) pc.degsum[c] = o_deg;
    if (pc.ein) pc.ein[c] = o_ein;
    if (pc.eout) pc.eout[c] = o_eout;
    if (pc.intra_density) pc.intra_density[c] = o_d;
    if (pc.contraction) pc.contraction[c] = o_contr;
    if (pc.expansion) pc.expansion[c] = o_exp;
    if (pc.conductance) pc.conductance[c] = o_cond;
    if (pc.q_term) pc.q_term[c] = o_q;
    if (pc.qds_term) pc.qds_term[c] = o_qds;
  }
  u64 fu[5] = {K, sein, seout, sD2, np};
  u128 fx[1] = {pen};
  double ff[5] = {qds_a, s_dens, s_contr, s_exp, s_cond};
  block_sum_fields(fu, fx, ff);
  if (threadIdx.x == 0) {
    ScorePart p;
    p.K = fu[0];
    p.sein = fu[1];
    p.seout = fu[2];
    p.sD2 = fu[3];
    p.np = fu[4];
    p.pen_lo = (u64)fx[0];
    p.pen_hi = (u64)(fx[0] >> 64);
    p.pad = 0;
    p.qds_a = ff[0];
    p.s_dens = ff[1];
    p.s_contr = ff[2];
    p.s_exp = ff[3];
    p.s_cond = ff[4];
    p.pad2[0] = p.pad2[1] = p.pad2[2] = 0;
    parts[blk] = p;
  }
}

__global__ __launch_bounds__(FBLOCK) void k_score_final1(int L, const u32* __restrict__ N, const u32* __restrict__ D,
                                                         const u32* __restrict__ I, const u32* __restrict__ NP,
                                                         const u64* __restrict__ PEN, double twom, PerComm pc,
                                                         ScorePart* __restrict__ parts) {
  score_final1_body(L, N, D, I, NP, PEN, twom, pc, parts, blockIdx.x, gridDim.x);
}

// device mirror of the public cq_score_result (same layout)
struct ScoreResultDev {
  int64_t n, m, K, num_pairs, sum_ein, sum_eout;
  uint64_t sum_degsum_sq;
  double Q, Qds, split_penalty;
  double mean_intra_edges, mean_intra_density, mean_contraction;
  double mean_inter_edges, mean_expansion, mean_conductance;
  uint32_t device_flags, weighted;
  double total_weight, sum_w_in, sum_w_out;
  uint32_t staging, reserved;
};

// staging reported in the result: the choice made on the device (ctl->mode) when there
// was one, else STAGE_BLOCKS for a column-blocked graph (blocked != 0), STAGE_ROWS_ONLY otherwise.
__device__ __forceinline__ u32 staging_of(const Ctl* ctl, u32 blocked) {
  return ctl->mode ? ctl->mode : (blocked ? STAGE_BLOCKS : STAGE_ROWS_ONLY);
}

__device__ void score_final2_body(int G, const ScorePart* __restrict__ parts, long long n, long long twom, long long ecap,
                                  Ctl* __restrict__ ctl, ScoreResultDev* __restrict__ out, u32 blocked) {
  u64 K = 0, sein = 0, seout = 0, sD2 = 0, np = 0;
  u128 pen = 0;
  double qds_a = 0, s_dens = 0, s_contr = 0, s_exp = 0, s_cond = 0;
  for (int b = 0; b < G; ++b) {
    const ScorePart p = parts[b];
    K += p.K; sein += p.sein; seout += p.seout; sD2 += p.sD2; np += p.np;
    pen += ((u128)p.pen_hi << 64) | p.pen_lo;
    qds_a += p.qds_a; s_dens += p.s_dens; s_contr += p.s_contr; s_exp += p.s_exp; s_cond += p.s_cond;
  }
  const long long m = twom / 2;
  ScoreResultDev r;
  r.n = n; r.m = m; r.K = (int64_t)K; r.num_pairs = (int64_t)np;
  r.sum_ein = (int64_t)sein; r.sum_eout = (int64_t)seout; r.sum_degsum_sq = sD2;
  // Eq. 8 summed over communities: sum_c E_c/m - (D_c/2m)^2 = (4 m sum_c E_c - sum_c D_c^2) / (4 m^2),
  // evaluated from exact integers with a single rounding of numerator and denominator.
  const long long qnum = 4ll * m * (long long)sein - (long long)sD2;
  r.Q = (double)qnum / (double)(4ull * (u64)m * (u64)m);
  const double p = unfix96(pen);
  r.split_penalty = p;
  r.Qds = qds_a - p;
  const double Kd = (double)K;
  r.mean_intra_edges = (double)sein / Kd;
  r.mean_intra_density = s_dens / Kd;
  r.mean_contraction = s_contr / Kd;
  r.mean_inter_edges = (double)seout / Kd;
  r.mean_expansion = s_exp / Kd;
  r.mean_conductance = s_cond / Kd;
  r.device_flags = ctl->flags | ((ecap > 0 && (long long)ctl->export_count > ecap) ? F_EXPORT : 0u);
  r.weighted = 0;
  r.total_weight = (double)m;
  r.sum_w_in = (double)sein;
  r.sum_w_out = (double)seout;
  r.staging = staging_of(ctl, blocked);
  r.reserved = 0;
  *out = r;
}

// Weighted final reduction (see group_one_w): per community the Eq. 8 and Eq. 9
// brackets and the six measures with weight sums, densities from the counts.
struct WScorePart {
  u64 K, sein, seout, sD2, np, penw_lo, penw_hi, wi_lo, wi_hi, wo_lo, wo_hi, pad;
  double q, qds_a, s_dens, s_contr, s_exp, s_cond, pad2[2];
};

__global__ __launch_bounds__(FBLOCK) void k_score_final1_w(int L, const u32* __restrict__ N, const u32* __restrict__ D,
                                                           const u32* __restrict__ I, const u32* __restrict__ NP,
                                                           const u64* __restrict__ SW, const u64* __restrict__ IW,
                                                           const u64* __restrict__ PENW, double W, PerComm pc,
                                                           WScorePart* __restrict__ parts) {
  const int G = gridDim.x, blk = blockIdx.x;
  const int R = (L + G - 1) / G;
  const int c0 = blk * R, c1 = min(L, c0 + R);
  u64 K = 0, sein = 0, seout = 0, sD2 = 0, np = 0;
  u128 penw = 0, swi2 = 0, swo = 0;
  double q = 0, qds_a = 0, s_dens = 0, s_contr = 0, s_exp = 0, s_cond = 0;
  for (int c = c0 + threadIdx.x; c < c1; c += FBLOCK) {
    const u32 nc = N[c];
    int64_t o_size = 0, o_deg = 0, o_ein = 0, o_eout = 0;
    double o_d = 0, o_contr = 0, o_exp = 0, o_cond = 0, o_q = 0, o_qds = 0, o_wi = 0, o_s = 0;
    if (nc > 0) {
      const u32 Dc = D[c], Ic = I[c];
      const u32 ein = Ic / 2u, eout = Dc - Ic;
      const u128 s128 = ((u128)SW[2 * (size_t)c + 1] << 64) | SW[2 * (size_t)c];
      const u128 i128 = ((u128)IW[2 * (size_t)c + 1] << 64) | IW[2 * (size_t)c];
      const u128 p128 = ((u128)PENW[2 * (size_t)c + 1] << 64) | PENW[2 * (size_t)c];
      const double sc = unfixw(s128);        // s(c)
      const double wi = 0.5 * unfixw(i128);  // w_in(c)
      const double wout = unfixw(s128 - i128);
      const double d = nc >= 2 ? (2.0 * (double)ein) / (double)((u64)nc * (u64)(nc - 1u)) : 0.0;
      const double tot = sc / (2.0 * W);
      const double tdc = tot * d;
      const double qa = wi / W * d - tdc * tdc;
      o_size = nc; o_deg = Dc; o_ein = ein; o_eout = eout;
      o_d = d;
      o_contr = 2.0 * wi / (double)nc;
      o_exp = wout / (double)nc;
      o_cond = sc > 0.0 ? wout / sc : 0.0;
      o_q = wi / W - tot * tot;
      o_qds = qa - unfix96(p128);
      o_wi = wi;
      o_s = sc;
      K += 1; sein += ein; seout += eout; sD2 += (u64)Dc * (u64)Dc; np += NP[c];
      penw += p128; swi2 += i128; swo += s128 - i128;
      q += o_q; qds_a += qa; s_dens += o_d; s_contr += o_contr; s_exp += o_exp; s_cond += o_cond;
    }
    if (pc.size) pc.size[c] = o_size;
    if (pc.degsum) pc.degsum[c] = o_deg;
    if (pc.ein) pc.ein[c] = o_ein;
    if (pc.eout) pc.eout[c] = o_eout;
    if (pc.intra_density) pc.intra_density[c] = o_d;
    if (pc.contraction) pc.contraction[c] = o_contr;
    if (pc.expansion) pc.expansion[c] = o_exp;
    if (pc.conductance) pc.conductance[c] = o_cond;
    if (pc.q_term) pc.q_term[c] = o_q;
    if (pc.qds_term) pc.qds_term[c] = o_qds;
    if (pc.w_in) pc.w_in[c] = o_wi;
    if (pc.strength) pc.strength[c] = o_s;
  }
  u64 fu[5] = {K, sein, seout, sD2, np};
  u128 fx[3] = {penw, swi2, swo};
  double ff[6] = {q, qds_a, s_dens, s_contr, s_exp, s_cond};
  block_sum_fields(fu, fx, ff);
  if (threadIdx.x == 0) {
    WScorePart p;
    p.K = fu[0];
    p.sein = fu[1];
    p.seout = fu[2];
    p.sD2 = fu[3];
    p.np = fu[4];
    p.penw_lo = (u64)fx[0];
    p.penw_hi = (u64)(fx[0] >> 64);
    p.wi_lo = (u64)fx[1];
    p.wi_hi = (u64)(fx[1] >> 64);
    p.wo_lo = (u64)fx[2];
    p.wo_hi = (u64)(fx[2] >> 64);
    p.pad = 0;
    p.q = ff[0];
    p.qds_a = ff[1];
    p.s_dens = ff[2];
    p.s_contr = ff[3];
    p.s_exp = ff[4];
    p.s_cond = ff[5];
    p.pad2[0] = p.pad2[1] = 0;
    parts[blk] = p;
  }
}

__global__ void k_score_final2_w(int G, const WScorePart* __restrict__ parts, long long n, long long twom, double W,
                                 long long ecap, Ctl* __restrict__ ctl, ScoreResultDev* __restrict__ out, u32 blocked) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  u64 K = 0, sein = 0, seout = 0, sD2 = 0, np = 0;
  u128 penw = 0, swi2 = 0, swo = 0;
  double q = 0, qds_a = 0, s_dens = 0, s_contr = 0, s_exp = 0, s_cond = 0;
  for (int b = 0; b < G; ++b) {
    const WScorePart p = parts[b];
    K += p.K; sein += p.sein; seout += p.seout; sD2 += p.sD2; np += p.np;
    penw += ((u128)p.penw_hi << 64) | p.penw_lo;
    swi2 += ((u128)p.wi_hi << 64) | p.wi_lo;
    swo += ((u128)p.wo_hi << 64) | p.wo_lo;
    q += p.q; qds_a += p.qds_a; s_dens += p.s_dens; s_contr += p.s_contr; s_exp += p.s_exp; s_cond += p.s_cond;
  }
  ScoreResultDev r;
  r.n = n; r.m = twom / 2; r.K = (int64_t)K; r.num_pairs = (int64_t)np;
  r.sum_ein = (int64_t)sein; r.sum_eout = (int64_t)seout; r.sum_degsum_sq = sD2;
  const double pen = unfix96(penw);
  r.Q = q;
  r.split_penalty = pen;
  r.Qds = qds_a - pen;
  const double Kd = (double)K;
  const double wi = 0.5 * unfixw(swi2), wout = unfixw(swo);
  r.mean_intra_edges = wi / Kd;
  r.mean_intra_density = s_dens / Kd;
  r.mean_contraction = s_contr / Kd;
  r.mean_inter_edges = wout / Kd;
  r.mean_expansion = s_exp / Kd;
  r.mean_conductance = s_cond / Kd;
  r.device_flags = ctl->flags | ((ecap > 0 && (long long)ctl->export_count > ecap) ? F_EXPORT : 0u);
  r.weighted = 1;
  r.total_weight = W;
  r.sum_w_in = wi;
  r.sum_w_out = wout;
  r.staging = staging_of(ctl, blocked);
  r.reserved = 0;
  *out = r;
}


__global__ void k_score_final2(int G, const ScorePart* __restrict__ parts, long long n, long long twom, long long ecap,
                               Ctl* __restrict__ ctl, ScoreResultDev* __restrict__ out, u32 blocked) {
  if (threadIdx.x == 0 && blockIdx.x == 0) score_final2_body(G, parts, n, twom, ecap, ctl, out, blocked);
}

// comparison final reduction ------------------------------------------------
struct CmpPart {
  u64 Ka, Kb, a11, X, Y, smax, xl_lo, xl_hi, sa_lo, sa_hi, sb_lo, sb_hi;
  double fsum, pad[3];
};

__global__ __launch_bounds__(FBLOCK) void k_cmp_final1(int La, int Lb, int Ga, const u32* __restrict__ A, const u32* __restrict__ B,
                                                       const u32* __restrict__ COLMAX, const u64* __restrict__ RA11,
                                                       const u32* __restrict__ RMAX, const double* __restrict__ RF,
                                                       const u64* __restrict__ RXL, double Nd, CmpPart* __restrict__ parts) {
  u64 Ka = 0, Kb = 0, a11 = 0, X = 0, Y = 0, smax = 0;
  u128 xl = 0, sa = 0, sb = 0;  // S, S_a, S_b (see CmpVis)
  double fsum = 0;
  if ((int)blockIdx.x < Ga) {  // rows: ground-truth communities
    const int R = (La + Ga - 1) / Ga;
    const int c0 = blockIdx.x * R, c1 = min(La, c0 + R);
    for (int i = c0 + threadIdx.x; i < c1; i += FBLOCK) {
      const u32 ai = A[i];
      if (ai == 0) continue;
      Ka += 1;
      a11 += RA11[i];
      smax += RMAX[i];
      X += (u64)ai * (u64)(ai - 1u) / 2u;
      xl += ((u128)RXL[2 * (size_t)i + 1] << 64) | RXL[2 * (size_t)i];
      fsum += (double)ai * RF[i];
      sa += fix96((double)ai / Nd * log((double)ai));
    }
  } else {  // columns: detected communities
    const int Gb = gridDim.x - Ga;
    const int R = (Lb + Gb - 1) / Gb;
    const int c0 = (blockIdx.x - Ga) * R, c1 = min(Lb, c0 + R);
    for (int j = c0 + threadIdx.x; j < c1; j += FBLOCK) {
      const u32 bj = B[j];
      if (bj == 0) continue;
      Kb += 1;
      smax += max(COLMAX[j], 1u);  // a non-empty column's largest cell holds at least one node
      Y += (u64)bj * (u64)(bj - 1u) / 2u;
      sb += fix96((double)bj / Nd * log((double)bj));
    }
  }
  u64 fu[6] = {Ka, Kb, a11, X, Y, smax};
  u128 fx[3] = {xl, sa, sb};
  double ff[1] = {fsum};
  block_sum_fields(fu, fx, ff);
  if (threadIdx.x == 0) {
    CmpPart p;
    p.Ka = fu[0];
    p.Kb = fu[1];
    p.a11 = fu[2];
    p.X = fu[3];
    p.Y = fu[4];
    p.smax = fu[5];
    p.xl_lo = (u64)fx[0]; p.xl_hi = (u64)(fx[0] >> 64);
    p.sa_lo = (u64)fx[1]; p.sa_hi = (u64)(fx[1] >> 64);
    p.sb_lo = (u64)fx[2]; p.sb_hi = (u64)(fx[2] >> 64);
    p.fsum = ff[0];
    p.pad[0] = p.pad[1] = p.pad[2] = 0;
    parts[blockIdx.x] = p;
  }
}

struct CmpResultDev {
  int64_t n, Ka, Kb, nnz, a11, a10, a01, a00, A;
  double VI, NMI, F, NVD, RI, ARI, JI;
  uint32_t device_flags, reserved;
};

__device__ __forceinline__ double i128_to_f64(__int128 v) {
  bool neg = v < 0;
  u128 a = neg ? (u128)(-v) : (u128)v;
  double d = ldexp((double)(u64)(a >> 64), 64) + (double)(u64)a;
  return neg ? -d : d;
}

__global__ void k_cmp_final2(int G, const CmpPart* __restrict__ parts, long long n, long long ecap, Ctl* __restrict__ ctl,
                             CmpResultDev* __restrict__ out, u32* __restrict__ wq) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  unsigned long long cells = 0;
  for (u32 q = 0; q < WQ_QUEUES; ++q) cells += *wq_sum(wq, q);
  u64 Ka = 0, Kb = 0, a11 = 0, X = 0, Y = 0, smax = 0;
  u128 xl = 0, sa = 0, sb = 0;
  double fsum = 0;
  for (int b = 0; b < G; ++b) {
    const CmpPart p = parts[b];
    Ka += p.Ka; Kb += p.Kb; a11 += p.a11; X += p.X; Y += p.Y; smax += p.smax;
    xl += ((u128)p.xl_hi << 64) | p.xl_lo;
    sa += ((u128)p.sa_hi << 64) | p.sa_lo;
    sb += ((u128)p.sb_hi << 64) | p.sb_lo;
    fsum += p.fsum;
  }
  const double Nd = (double)n;
  const u64 A = (u64)n * (u64)(n - 1) / 2u;
  CmpResultDev r;
  r.n = n; r.Ka = (int64_t)Ka; r.Kb = (int64_t)Kb; r.nnz = (int64_t)cells;
  r.a11 = (int64_t)a11;
  r.a10 = (int64_t)(X - a11);
  r.a01 = (int64_t)(Y - a11);
  r.a00 = (int64_t)(A - X - Y + a11);
  r.A = (int64_t)A;
  // combined in fixed point before the one conversion (see CmpVis).  A side with one
  // community has entropy 0 and shares no information: exactly, from the counts.
  const double logN = log(Nd);
  r.VI = -unfix96(2 * xl - sa - sb);
  const double ha = Ka == 1 ? 0.0 : logN - unfix96(sa);  // H(C)
  const double hb = Kb == 1 ? 0.0 : logN - unfix96(sb);  // H(C')
  const double mi = (Ka == 1 || Kb == 1) ? 0.0 : unfix96(xl - sa - sb) + logN;
  const double den = ha + hb;
  r.NMI = den != 0.0 ? 2.0 * mi / den : 1.0;
  r.F = fsum / Nd;
  r.NVD = 1.0 - (double)smax / (2.0 * Nd);
  r.RI = (double)(a11 + (A - X - Y + a11)) / (double)A;
  // Eq. 6 with M = (a11+a10)(a11+a01)/A, numerator and denominator scaled by 2A:
  // ARI = (2 A a11 - 2 X Y) / (A (X + Y) - 2 X Y), exact in 128-bit integers.
  const __int128 XY = (__int128)X * (__int128)Y;
  const __int128 anum = 2 * (__int128)A * (__int128)a11 - 2 * XY;
  const __int128 aden = (__int128)A * (__int128)(X + Y) - 2 * XY;
  r.ARI = aden != 0 ? i128_to_f64(anum) / i128_to_f64(aden) : 1.0;
  const u64 jden = a11 + (X - a11) + (Y - a11);
  r.JI = jden != 0 ? (double)a11 / (double)jden : 1.0;
  r.device_flags = ctl->flags | ((ecap > 0 && (long long)ctl->export_count > ecap) ? F_EXPORT : 0u);
  r.reserved = 0;
  *out = r;
}

// ---------------------------------------------------------------------------
// Batched scoring: many (graph, partition) tasks per launch.  Every stage of the
// scoring path runs as one launch over the work of all tasks; blocks find their task
// through prefix tables built by the host plan.  Tasks that share a graph are grouped
// (up to BATCH_FUSE partitions), and the edge pass reads that graph's col_idx once for
// the whole group.  Batched tasks use LDS-private histograms and 16-bit labels
// (num_labels <= 16384).
constexpr int BATCH_FUSE = 4;
constexpr int BG_UNROLL = 4;  // entries per thread in flight in the batched edge pass

struct TaskDev {
  const int32_t* labels;
  const int32_t* perm;
  const int32_t* rp;
  const int32_t* col;
  long long nnz;
  int n, L, chunk, W, G;
  int lst;  // labx stride: the labels go to lane p of the task's group's interleaved words (GroupDev::il)
  Ctl* ctl;
  u32 *N, *D, *start, *order, *I, *NP;
  u64* PEN;
  u32* loc;
  u32 *HN, *HD;
  uint16_t* labx;
  uint16_t* CB;
  ScorePart* parts;
  ScoreResultDev* out;
};

struct GroupDev {
  const int32_t* rp;
  const int32_t* col;
  int n, np;
  int task[BATCH_FUSE];
  // per stored node: the group's partitions' labels, 16 bits each (partition p at bits 16p),
  // written by the node pass; the edge pass reads a neighbour's labels in every partition
  // with one load (random 2-byte reads are L2 requests, and their rate is what the edge
  // pass spends)
  unsigned long long* il;
};

// largest i in [0, cnt) with pre[i] <= x (pre non-decreasing, pre[0] == 0)
__device__ __forceinline__ int find_seg(const u32* __restrict__ pre, int cnt, u32 x) {
  int lo = 0, hi = cnt - 1;
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (pre[mid] <= x) lo = mid; else hi = mid - 1;
  }
  return lo;
}

__global__ void k_b_setup(int T, const TaskDev* __restrict__ td, u32* __restrict__ wq) {
  const int t = blockIdx.x;
  if (t < T) {
    u32* c = reinterpret_cast<u32*>(td[t].ctl);
    for (int i = threadIdx.x; i < (int)(sizeof(Ctl) / 4); i += blockDim.x) c[i] = 0;
  }
  if (t == 0)
    for (u32 i = threadIdx.x; i < 2 * WQ_WORDS; i += blockDim.x) wq[i] = 0;  // both group passes' queues
}

// Node pass over every task's chunks.  Workgroup b runs on XCD b % 8 and takes entry
// b / 8 of that XCD's list, so that the labels a task reads at random (in the caller's
// order, through the graph's permutation) are pulled into one XCD's L2.  Per XCD, T list
// entries: XW the chunk prefix (T + 1 values, padded with the total), XT the task, then
// its first chunk (bit 31: the entry takes every 8th chunk of the task, else consecutive
// ones).
__global__ __launch_bounds__(1024) void k_b_node(const TaskDev* __restrict__ td, const u32* __restrict__ XW,
                                                 const u32* __restrict__ XT, int T) {
  const u32 x = blockIdx.x % 8u, i = blockIdx.x / 8u;
  const u32* pre = XW + (size_t)x * (T + 1);
  if (i >= pre[T]) return;
  const int j = find_seg(pre, T, i);
  const int t = (int)XT[(size_t)x * T + j];
  const u32 fo = XT[(size_t)8 * T + (size_t)x * T + j];
  const u32 blk = (fo & 0x7FFFFFFFu) + ((fo >> 31) ? 8u : 1u) * (i - pre[j]);
  const TaskDev& d = td[t];
  node_priv_body<true, uint16_t>(d.n, d.labels, d.perm, d.rp, d.L, d.chunk, d.HN, d.HD, d.loc, d.labx, d.ctl, (int)blk,
                                 0, d.L, d.lst);
}

__global__ __launch_bounds__(256) void k_b_colscan(const TaskDev* __restrict__ td, const u32* __restrict__ Lpre, int T) {
  const u32 gid = blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= Lpre[T]) return;
  const int t = find_seg(Lpre, T, gid);
  const TaskDev& d = td[t];
  colscan_body<true, true>(d.W, d.L, d.HN, d.HD, d.N, d.D, (int)(gid - Lpre[t]));
}

__global__ __launch_bounds__(1024) void k_b_scan_order(const TaskDev* __restrict__ td) {
  const TaskDev& d = td[blockIdx.x];
  scan_order_body(d.L, d.N, d.D, d.start, d.order, d.ctl);
}

// Kpre[t] = number of non-empty communities of tasks before t; Kpre[T] = total
__global__ __launch_bounds__(1024) void k_b_kprefix(const TaskDev* __restrict__ td, int T, u32* __restrict__ Kpre) {
  __shared__ u32 s_w[SCAN_THREADS / 64];
  __shared__ u32 s_carry;
  if (threadIdx.x == 0) s_carry = 0;
  __syncthreads();
  for (int b = 0; b < T; b += SCAN_THREADS) {
    const int i = b + threadIdx.x;
    const u32 x = i < T ? td[i].ctl->K : 0u;
    u32 total;
    const u32 ex = block_excl_scan_1024(x, s_w, &total);
    const u32 carry = s_carry;
    if (i < T) Kpre[i] = carry + ex;
    __syncthreads();
    if (threadIdx.x == 0) s_carry = carry + total;
    __syncthreads();
  }
  if (threadIdx.x == 0) Kpre[T] = s_carry;
}

// Edge pass for a group of partitions of one graph: every col_idx entry is read once
// and the neighbour's label of each partition goes to that partition's segment.
// Workgroup b runs on XCD b % 8 (workgroups are handed to the XCDs in turn) and takes
// tile b / 8 of that XCD's list: a graph's tiles run on one XCD, so the neighbour labels
// they read at random stay in that XCD's L2, except for graphs large enough to unbalance
// the XCDs, whose tiles are dealt to all eight in turn.  Per XCD, ngroups list entries:
// XRB the tile prefix (ngroups + 1 values, padded with the total), XG the group, XO its
// first tile (bit 31: the entry takes every 8th tile of the group, else consecutive ones).
template <int R>
__global__ __launch_bounds__(R) void k_b_gather(const GroupDev* __restrict__ gd, const u32* __restrict__ XRB,
                                                const u32* __restrict__ XG, int ngroups, const TaskDev* __restrict__ td) {
  __shared__ int s_rs[R + 1];
  __shared__ u32 s_base[BATCH_FUSE][R];
  const u32 x = blockIdx.x % 8u, i = blockIdx.x / 8u;
  const u32* pre = XRB + (size_t)x * (ngroups + 1);
  if (i >= pre[ngroups]) return;
  const int j = find_seg(pre, ngroups, i);
  const int k = (int)XG[(size_t)x * ngroups + j];
  const u32 xo = XG[(size_t)8 * ngroups + (size_t)x * ngroups + j];
  const u32 tile = (xo & 0x7FFFFFFFu) + ((xo >> 31) ? 8u : 1u) * (i - pre[j]);
  const GroupDev grp = gd[k];
  const int tid = threadIdx.x;
  const long long r0 = (long long)tile * R;
  const int rows = (int)min((long long)R, (long long)grp.n - r0);
  const unsigned long long* __restrict__ il = grp.il;
  if (tid < rows) {
    const long long u = r0 + tid;
    s_rs[tid] = grp.rp[u];
    const unsigned long long own = il[u];  // the row's label in every partition
#pragma unroll
    for (int p = 0; p < BATCH_FUSE; ++p) {
      if (p < grp.np) {
        const TaskDev& d = td[grp.task[p]];
        const uint16_t c = (uint16_t)(own >> (16 * p));
        const u32 lu = d.loc[u];
        u32 base = SENT;
        if (c != LabelT<uint16_t>::SENTINEL && lu != SENT) base = d.start[c] + d.HD[(size_t)(u / d.chunk) * d.L + c] + lu;
        s_base[p][tid] = base;
      }
    }
  }
  if (tid == 0) s_rs[rows] = grp.rp[r0 + rows];
  __syncthreads();
  uint16_t* cb[BATCH_FUSE];
#pragma unroll
  for (int p = 0; p < BATCH_FUSE; ++p) cb[p] = p < grp.np ? td[grp.task[p]].CB : nullptr;
  const int e0 = s_rs[0], e1 = s_rs[rows];
  // BG_UNROLL entries per thread at a time: their row searches (a fixed number of steps)
  // and their loads are all issued before the first label is used
  int top = 0;  // largest power of two below rows (0 for one row)
  if (rows > 1) top = 1 << (31 - __clz(rows - 1));
  for (int eb = e0 + tid; eb < e1; eb += BG_UNROLL * R) {
    int lo[BG_UNROLL], v[BG_UNROLL];
#pragma unroll
    for (int k = 0; k < BG_UNROLL; ++k) {
      const int e = min(eb + k * R, e1 - 1);  // in bounds; masked below
      int l = 0;  // last row r with s_rs[r] <= e
      for (int st = top; st > 0; st >>= 1)
        if (l + st < rows && s_rs[l + st] <= e) l += st;
      lo[k] = l;
      v[k] = grp.col[e];
    }
    unsigned long long w[BG_UNROLL];
#pragma unroll
    for (int k = 0; k < BG_UNROLL; ++k) w[k] = il[v[k]];  // the neighbour's labels in every partition: one load
#pragma unroll
    for (int k = 0; k < BG_UNROLL; ++k) {
      const int e = eb + k * R;
      if (e < e1) {
        const u32 off = (u32)(e - s_rs[lo[k]]);
#pragma unroll
        for (int p = 0; p < BATCH_FUSE; ++p) {
          if (p < grp.np) {
            const u32 b = s_base[p][lo[k]];
            if (b != SENT) cb[p][b + off] = (uint16_t)(w[k] >> (16 * p));
          }
        }
      }
    }
  }
}

// The group pass's items as one list: item i (Kpre[t] <= i < Kpre[t+1]) is group
// g = order_t[i - Kpre[t]] of task t, written as ((t << 14) | g, start_t[g], D_t[g], 0)
// (groups < 16384 in a batch), so that the persistent pass reaches a community's segment
// with one load after its ticket instead of a search over Kpre and two dependent loads.
__global__ __launch_bounds__(256) void k_b_items(const TaskDev* __restrict__ td, const u32* __restrict__ Kpre, int T,
                                                 uint4* __restrict__ items) {
  const u32 total = Kpre[T];
  for (u32 i = blockIdx.x * blockDim.x + threadIdx.x; i < total; i += gridDim.x * blockDim.x) {
    const int t = find_seg(Kpre, T, i);
    const TaskDev& d = td[t];
    const u32 g = d.order[i - Kpre[t]];
    items[i] = make_uint4(((u32)t << 14) | g, d.start[g], d.D[g], 0u);
  }
}

// Persistent group pass over the communities of every task (per-XCD work queues, wq_next),
// in workgroups of NT threads, as a single call with the same label count: one launch
// (NT = GBLOCK_SMALL, small != 0) takes the communities of tasks with at most SMALL_L_MAX
// label ids and skips the others, a second one (NT = GBLOCK_DIRECT) the rest.
template <int NT>
__global__ __launch_bounds__(NT, 8) void k_b_groups(const TaskDev* __restrict__ td, const u32* __restrict__ Kpre, int T,
                                                    u32* __restrict__ wq, u32 lds_words, const uint4* __restrict__ items,
                                                    int small) {
  __shared__ u32 s_item;
  __shared__ uint4 s_it;
  const u32 total = Kpre[T];
  u32 q = blockIdx.x % WQ_QUEUES, left = WQ_QUEUES;  // thread 0's queue state (see wq_next)
  for (;;) {
    if (threadIdx.x == 0) {
      const u32 it = wq_next(wq, total, q, left);
      s_item = it;
      s_it = it < total ? items[it] : make_uint4(0u, 0u, 0u, 0u);
    }
    __syncthreads();
    const u32 item = s_item;
    const uint4 x = s_it;
    __syncthreads();
    if (item >= total) break;
    const int t = (int)(x.x >> 14);
    const TaskDev& d = td[t];
    if (((u32)d.L <= SMALL_L_MAX) != (small != 0)) continue;  // the other launch's community
    const u32 g = x.x & 0x3FFFu;
    ScoreVis vis;
    vis.N = d.N;
    vis.twom = (double)d.nnz;
    vis.I = d.I;
    vis.NP = d.NP;
    vis.PEN = d.PEN;
    vis.eci = nullptr;
    vis.ecj = nullptr;
    vis.ecnt = nullptr;
    vis.ecap = 0;
    vis.ctl = d.ctl;
    group_one<ScoreVis, uint16_t, NT>(d.CB, x.y, x.z, g, (u32)d.L, lds_words, vis, d.ctl);
  }
}

__global__ __launch_bounds__(FBLOCK) void k_b_final1(const TaskDev* __restrict__ td, const u32* __restrict__ Gpre, int T) {
  const int t = find_seg(Gpre, T, blockIdx.x);
  const TaskDev& d = td[t];
  PerComm pc = {};
  score_final1_body(d.L, d.N, d.D, d.I, d.NP, d.PEN, (double)d.nnz, pc, d.parts, (int)(blockIdx.x - Gpre[t]), d.G);
}

__global__ void k_b_final2(const TaskDev* __restrict__ td, int T) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= T) return;
  const TaskDev& d = td[t];
  score_final2_body(d.G, d.parts, d.n, d.nnz, 0, d.ctl, d.out, 0u);
}

}  // namespace cq
