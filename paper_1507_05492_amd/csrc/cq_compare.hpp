// Comparison of two partitions with at most 65,535 labels each (Section II-A): the
// contingency table n_ij = |c_i ∩ c'_j| built by label bands, and its reduction to the
// per-row quantities the final pass combines into VI, NMI, F, NVD, RI, ARI and JI
// (Eqs. (1)-(7)).
//
// The ground-truth labels are cut into bands: runs of consecutive label ids holding about
// T nodes (and at most CB_ROWS labels); the band sizes and their places follow from the
// label sizes alone.  A pass over chunks of nodes writes every node as one 32-bit word
// (label - first label of its band) << 16 | detected label into its band's range: a
// chunk counts its nodes per band in LDS, claims a run of places in each band with one
// atomic, lays its words out in LDS band by band, and writes them in that order, so the
// stores of a wave go to a few runs of consecutive words rather than to 64 scattered
// places.  Then a persistent workgroup takes a whole band: it counts the band's cells
// (row, detected label) in an LDS hash table and visits every cell once, keeping each
// row's sums and maxima in LDS, and writes the rows' results.  A band whose distinct cells
// overflow the table is split into residue classes of the detected label (mod 2, 4, ...),
// each counted and visited on its own; cells of different classes are different cells, so
// every cell is still visited exactly once.
//
// All sums are over integers or exact fixed point, so the results do not depend on the
// order of the atomics and equal those of the segment-per-community path bit for bit.
#pragma once

namespace cq {

constexpr int CB_ROWS = 128;          // labels per band at most (rows of a band; the row part of a word has 8 bits)
constexpr int CB_PER = 16;            // labels per thread and round in k_cmp_bands
constexpr int CC_THREADS = 512;       // k_cmp_cells workgroup
constexpr int CC_LOG2_SLOTS = 13;
constexpr u32 CC_SLOTS = 1u << CC_LOG2_SLOTS;  // LDS hash slots (key and count words)
constexpr u32 CC_PROBE = 64;          // a key that finds no place within this many slots splits its class
constexpr int CC_SUB = 8;             // counters per row for the row's dominant detected label
constexpr u32 CC_JUMP = 2;            // a class that overflows is split into up to 2^CC_JUMP classes
constexpr int CC_STACK = 64;          // pending residue classes (depth first)
constexpr int CC_BATCH = 8;           // band words each thread loads at once
constexpr u32 CMP_BAD_B = 0xFFFFu;    // detected label outside [0, Lb)

// A flag in LDS that other threads of the workgroup may set: read as a workgroup-scope
// atomic, which stays an LDS read (a volatile access through a generic pointer would
// become a flat load that also waits for the thread's outstanding global loads).
__device__ __forceinline__ u32 lds_flag(u32* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// Label histograms of both partitions in one pass, when both label spaces fit one LDS
// table together: row blockIdx.x of HA (La counters) and HB (Lb counters).  Labels out
// of range are flagged (F_LABEL) and not counted.
constexpr int H2_NPT = 16;  // labels of each side per thread and round
__global__ __launch_bounds__(1024) void k_hist2_priv(int n, const int32_t* __restrict__ la, int La,
                                                     const int32_t* __restrict__ lb, int Lb, u32* __restrict__ HA,
                                                     u32* __restrict__ HB, Ctl* __restrict__ ctl) {
  extern __shared__ u32 s_h2[];
  u32* sa = s_h2;
  u32* sb = s_h2 + La;
  __shared__ u32 s_bad;
  for (int i = threadIdx.x; i < La + Lb; i += 1024) s_h2[i] = 0;
  if (threadIdx.x == 0) s_bad = 0;
  __syncthreads();
  u32 bad = 0;
  for (long long base = (long long)blockIdx.x * 1024 * H2_NPT; base < n; base += (long long)gridDim.x * 1024 * H2_NPT) {
    int a[H2_NPT], b[H2_NPT];
#pragma unroll
    for (int k = 0; k < H2_NPT; ++k) {
      const long long u = base + threadIdx.x + (long long)k * 1024;
      a[k] = u < n ? la[u] : -1;
      b[k] = u < n ? lb[u] : -1;
      if (u < n) bad |= ((u32)a[k] >= (u32)La) | ((u32)b[k] >= (u32)Lb);
    }
#pragma unroll
    for (int k = 0; k < H2_NPT; ++k) {
      if ((u32)a[k] < (u32)La) atomicAdd(&sa[a[k]], 1u);
      if ((u32)b[k] < (u32)Lb) atomicAdd(&sb[b[k]], 1u);
    }
  }
  if (bad) s_bad = 1;
  __syncthreads();
  for (int c = threadIdx.x; c < La; c += 1024) HA[(size_t)blockIdx.x * La + c] = sa[c];
  for (int c = threadIdx.x; c < Lb; c += 1024) HB[(size_t)blockIdx.x * Lb + c] = sb[c];
  if (threadIdx.x == 0 && s_bad) atomicOr(&ctl->flags, F_LABEL);
}

// Clears the control block, the work queues and (Lb > 0) the column maxima in one launch.
__global__ __launch_bounds__(256) void k_cmp_clear(u32* __restrict__ ctl_words, int nctl, u32* __restrict__ wq,
                                                   u32* __restrict__ COLMAX, int Lb) {
  const int stride = gridDim.x * blockDim.x;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < nctl + (int)WQ_WORDS + Lb; i += stride) {
    if (i < nctl) ctl_words[i] = 0;
    else if (i < nctl + (int)WQ_WORDS) wq[i - nctl] = 0;
    else COLMAX[i - nctl - (int)WQ_WORDS] = 0;
  }
}

// Label totals of both partitions from the per-workgroup rows of k_hist2_priv in one
// launch: blocks [0, ga) take the ground-truth labels, the others the detected ones.
__global__ __launch_bounds__(CS_LABELS * CS_GROUPS) void k_cmp_totals(int W, int La, int Lb, int ga,
                                                                      const u32* __restrict__ HA,
                                                                      const u32* __restrict__ HB, u32* __restrict__ A,
                                                                      u32* __restrict__ B) {
  __shared__ u32 s_n[CS_GROUPS][CS_LABELS];
  const bool side_a = (int)blockIdx.x < ga;
  const int L = side_a ? La : Lb;
  const u32* H = side_a ? HA : HB;
  u32* N = side_a ? A : B;
  const int lane = threadIdx.x % CS_LABELS, grp = threadIdx.x / CS_LABELS;
  const int c = (side_a ? (int)blockIdx.x : (int)blockIdx.x - ga) * CS_LABELS + lane;
  const int per = (W + CS_GROUPS - 1) / CS_GROUPS;
  const int w0 = min(W, grp * per), w1 = min(W, w0 + per);
  u32 sn = 0;
  if (c < L)
    for (int w = w0; w < w1; ++w) sn += H[(size_t)w * L + c];
  s_n[grp][lane] = sn;
  __syncthreads();
  if (c < L && grp == 0) {
    u32 t = 0;
    for (int i = 0; i < CS_GROUPS; ++i) t += s_n[i][lane];
    N[c] = t;
  }
}

// Bands of ground-truth labels from their sizes A (one workgroup).  Band k holds the
// labels SBA[k] .. SBA[k+1]-1 and the nodes SBS[k] .. SBS[k+1]-1 of the band words; a band
// ends after label a when the running node count passes a multiple of T inside a, after
// every CB_ROWS-th label, and at the last label.  sbk[a] = band << 8 | (a - SBA[band]).
// CUR[k] = SBS[k] (the claim cursors of k_cmp_part), SZB[k] = the band's node count,
// BORD = the non-empty bands by decreasing floor(log2 size), ctl->K = their number.
__global__ __launch_bounds__(1024) void k_cmp_bands(int La, const u32* __restrict__ A, u32 T, u32* __restrict__ sbk,
                                                    u32* __restrict__ SBA, u32* __restrict__ SBS, u32* __restrict__ SZB,
                                                    u32* __restrict__ CUR, u32* __restrict__ BORD, Ctl* __restrict__ ctl) {
  __shared__ u32 s_wtot[16], s_etot[16];
  __shared__ u32 s_carry, s_ecarry;
  __shared__ u32 s_bcnt[33], s_boff[33];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  if (tid == 0) {
    s_carry = 0;
    s_ecarry = 0;
    SBA[0] = 0;
    SBS[0] = 0;
  }
  if (tid < 33) s_bcnt[tid] = 0;
  __syncthreads();
  for (int base = 0; base < La; base += 1024 * CB_PER) {
    const int c0 = base + tid * CB_PER;
    u32 cnt[CB_PER];
    u32 sum = 0;
#pragma unroll
    for (int k = 0; k < CB_PER; ++k) {
      cnt[k] = c0 + k < La ? A[c0 + k] : 0u;
      sum += cnt[k];
    }
    const u32 incl = wave_incl_scan(sum);
    if (lane == 63) s_wtot[wv] = incl;
    __syncthreads();
    u32 P = s_carry + incl - sum;  // nodes of the labels before c0
    for (int i = 0; i < wv; ++i) P += s_wtot[i];
    u32 ends = 0, ne = 0;
    {
      u32 Pk = P;
#pragma unroll
      for (int k = 0; k < CB_PER; ++k) {
        const int a = c0 + k;
        const u32 Q = Pk + cnt[k];
        if (a < La && (Q / T != Pk / T || (a + 1) % CB_ROWS == 0 || a == La - 1)) {
          ends |= 1u << k;
          ++ne;
        }
        Pk = Q;
      }
    }
    const u32 eincl = wave_incl_scan(ne);
    if (lane == 63) s_etot[wv] = eincl;
    __syncthreads();
    u32 band = s_ecarry + eincl - ne;  // bands ended before label c0 = band of c0
    for (int i = 0; i < wv; ++i) band += s_etot[i];
#pragma unroll
    for (int k = 0; k < CB_PER; ++k) {
      const int a = c0 + k;
      P += cnt[k];
      if (a < La) {
        sbk[a] = band;
        if (ends & (1u << k)) {
          ++band;
          SBA[band] = (u32)a + 1u;
          SBS[band] = P;
        }
      }
    }
    __syncthreads();
    if (tid == 0) {
      u32 t = s_carry, e = s_ecarry;
      for (int i = 0; i < 16; ++i) {
        t += s_wtot[i];
        e += s_etot[i];
      }
      s_carry = t;
      s_ecarry = e;
    }
    __syncthreads();
  }
  // every band's first label and place is written: band numbers become band << 8 | row
  const u32 nb = s_ecarry;
  for (int a = tid; a < La; a += 1024) {
    const u32 k = sbk[a];
    sbk[a] = (k << 8) | ((u32)a - SBA[k]);
  }
  for (u32 k = tid; k < nb; k += 1024) {
    const u32 sz = SBS[k + 1] - SBS[k];
    SZB[k] = sz;
    CUR[k] = SBS[k];
    if (sz) atomicAdd(&s_bcnt[size_bucket(sz)], 1u);
  }
  __syncthreads();
  if (tid == 0) {
    u32 off = 0;
    for (int c = 32; c >= 0; --c) {
      s_boff[c] = off;
      off += s_bcnt[c];
    }
    ctl->K = off;
  }
  __syncthreads();
  for (u32 k = tid; k < nb; k += 1024) {
    const u32 sz = SZB[k];
    if (sz) BORD[atomicAdd(&s_boff[size_bucket(sz)], 1u)] = k;
  }
}

constexpr int CP_THREADS = 1024;
constexpr int CP_NPT = 20;                        // nodes per thread (at 10M nodes: 489 workgroups, two waves at one per CU)
constexpr int CP_CHUNK = CP_THREADS * CP_NPT;     // nodes per workgroup of k_cmp_part

// Exclusive scan of v[0, m) in LDS by one 1024-thread workgroup (m <= 4 * 1024); returns
// the total.  Each thread takes four consecutive entries.
__device__ __forceinline__ u32 block_excl_scan4(u32* v, int m, u32* s_w) {
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int i0 = tid * 4;
  u32 x[4], sum = 0;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    x[k] = i0 + k < m ? v[i0 + k] : 0u;
    sum += x[k];
  }
  const u32 incl = wave_incl_scan(sum);
  if (lane == 63) s_w[wv] = incl;
  __syncthreads();
  u32 run = incl - sum, tot = 0;
  for (int i = 0; i < CP_THREADS / 64; ++i) {
    if (i < wv) run += s_w[i];
    tot += s_w[i];
  }
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    if (i0 + k < m) v[i0 + k] = run;
    run += x[k];
  }
  __syncthreads();
  return tot;
}

// Writes every node of chunk blockIdx.x (rounds * CP_CHUNK nodes) into its band (see the
// file comment): the chunk counts its nodes per band, claims one run of places in each band
// it has nodes of, then, one round of CP_CHUNK nodes at a time, lays the round's words out
// in LDS band by band and writes them in that order.  Nodes whose ground-truth label is
// out of range are left out (the label histogram flags them); a detected label out of
// range is written as CMP_BAD_B.  nb bands (nb <= 4096).
__global__ __launch_bounds__(CP_THREADS) void k_cmp_part(int n, const int32_t* __restrict__ la,
                                                         const int32_t* __restrict__ lb, int La, int Lb,
                                                         const u32* __restrict__ sbk, int nb, int rounds,
                                                         u32* __restrict__ CUR, u32* __restrict__ E) {
  __shared__ u32 s_buf[CP_CHUNK];
  __shared__ uint16_t s_bid[CP_CHUNK];
  __shared__ u32 s_w[CP_THREADS / 64];
  extern __shared__ u32 s_dyn[];
  u32* s_run = s_dyn;           // the chunk's nodes per band, then the next global place of its run
  u32* s_rc = s_dyn + nb;       // the round's nodes per band, then their first place in s_buf
  const int tid = threadIdx.x;
  for (int i = tid; i < nb; i += CP_THREADS) s_run[i] = 0;
  if (rounds == 1) {
    // one round: the round's counts are the chunk's counts, so the labels are read once
    for (int i = tid; i < nb; i += CP_THREADS) s_rc[i] = 0;
    __syncthreads();
    const long long u0 = (long long)blockIdx.x * CP_CHUNK;
    u32 word[CP_NPT], key[CP_NPT], rank[CP_NPT];
#pragma unroll
    for (int k = 0; k < CP_NPT; ++k) {
      const long long u = u0 + tid + (long long)k * CP_THREADS;
      int a = -1, b = 0;
      if (u < n) {
        a = la[u];
        b = lb[u];
      }
      key[k] = (u32)a < (u32)La ? (u32)a : 0xFFFFFFFFu;
      word[k] = (u32)b < (u32)Lb ? (u32)b : CMP_BAD_B;
    }
#pragma unroll
    for (int k = 0; k < CP_NPT; ++k)
      if (key[k] != 0xFFFFFFFFu) key[k] = sbk[key[k]];
#pragma unroll
    for (int k = 0; k < CP_NPT; ++k)
      if (key[k] != 0xFFFFFFFFu) rank[k] = atomicAdd(&s_rc[key[k] >> 8], 1u);
    __syncthreads();
    for (int i = tid; i < nb; i += CP_THREADS) {
      const u32 c = s_rc[i];
      s_run[i] = c ? atomicAdd(&CUR[i], c) : 0u;  // one claim per band the chunk has nodes of
    }
    const u32 total = block_excl_scan4(s_rc, nb, s_w);
#pragma unroll
    for (int k = 0; k < CP_NPT; ++k) {
      if (key[k] != 0xFFFFFFFFu) {
        const u32 band = key[k] >> 8;
        const u32 p = s_rc[band] + rank[k];
        s_buf[p] = ((key[k] & 0xFFu) << 16) | word[k];
        s_bid[p] = (uint16_t)band;
      }
    }
    __syncthreads();
    for (u32 p = tid; p < total; p += CP_THREADS) {
      const u32 band = s_bid[p];
      E[s_run[band] + (p - s_rc[band])] = s_buf[p];
    }
    return;
  }
  __syncthreads();
  const long long c0 = (long long)blockIdx.x * rounds * CP_CHUNK;
  for (int r = 0; r < rounds; ++r) {
    const long long u0 = c0 + (long long)r * CP_CHUNK;
    u32 key[CP_NPT];
#pragma unroll
    for (int k = 0; k < CP_NPT; ++k) {
      const long long u = u0 + tid + (long long)k * CP_THREADS;
      const int a = u < n ? la[u] : -1;
      key[k] = (u32)a < (u32)La ? (u32)a : 0xFFFFFFFFu;
    }
#pragma unroll
    for (int k = 0; k < CP_NPT; ++k)
      if (key[k] != 0xFFFFFFFFu) atomicAdd(&s_run[sbk[key[k]] >> 8], 1u);
  }
  __syncthreads();
  for (int i = tid; i < nb; i += CP_THREADS) {
    const u32 c = s_run[i];
    s_run[i] = c ? atomicAdd(&CUR[i], c) : 0u;  // one claim per band the chunk has nodes of
  }
  for (int r = 0; r < rounds; ++r) {
    const long long u0 = c0 + (long long)r * CP_CHUNK;
    for (int i = tid; i < nb; i += CP_THREADS) s_rc[i] = 0;
    __syncthreads();  // also: the claims are in s_run, the previous round's writes have read s_buf
    u32 word[CP_NPT], key[CP_NPT], rank[CP_NPT];
#pragma unroll
    for (int k = 0; k < CP_NPT; ++k) {
      const long long u = u0 + tid + (long long)k * CP_THREADS;
      int a = -1, b = 0;
      if (u < n) {
        a = la[u];
        b = lb[u];
      }
      key[k] = (u32)a < (u32)La ? (u32)a : 0xFFFFFFFFu;
      word[k] = (u32)b < (u32)Lb ? (u32)b : CMP_BAD_B;
    }
#pragma unroll
    for (int k = 0; k < CP_NPT; ++k)
      if (key[k] != 0xFFFFFFFFu) key[k] = sbk[key[k]];
#pragma unroll
    for (int k = 0; k < CP_NPT; ++k)
      if (key[k] != 0xFFFFFFFFu) rank[k] = atomicAdd(&s_rc[key[k] >> 8], 1u);
    __syncthreads();
    const u32 total = block_excl_scan4(s_rc, nb, s_w);  // s_rc: first place of each band's words in s_buf
#pragma unroll
    for (int k = 0; k < CP_NPT; ++k) {
      if (key[k] != 0xFFFFFFFFu) {
        const u32 band = key[k] >> 8;
        const u32 p = s_rc[band] + rank[k];
        s_buf[p] = ((key[k] & 0xFFu) << 16) | word[k];
        s_bid[p] = (uint16_t)band;
      }
    }
    __syncthreads();
    for (u32 p = tid; p < total; p += CP_THREADS) {
      const u32 band = s_bid[p];
      E[s_run[band] + (p - s_rc[band])] = s_buf[p];
    }
    __syncthreads();
    // the round's runs are written: advance each band's place by its words of this round
    for (int i = tid; i < nb; i += CP_THREADS) {
      const u32 next = i + 1 < nb ? s_rc[i + 1] : total;
      s_run[i] += next - s_rc[i];
    }
    __syncthreads();  // s_rc is read above before the next round clears it
  }
}

// One band at a time per workgroup (bands by decreasing size from the work queues).
// A = |c_i|, B = |c'_j|; outputs per ground-truth label i: RA11 = Σ_j C(n_ij, 2),
// RMAX = max_j n_ij, RF = max_j 2 n_ij / (|c_i| + |c'_j|) (Eq. (3)), RXL = Σ_j fix96 of
// (n_ij / N) log n_ij; per detected label: COLMAX = max_i n_ij (cells of one node are left
// to the final pass, which counts 1 for every non-empty column); non-zero cells are
// summed per work queue; optional export of (i, j, n_ij).
__global__ __launch_bounds__(CC_THREADS, 4) void k_cmp_cells(const u32* __restrict__ E, const u32* __restrict__ SBS,
                                                          const u32* __restrict__ SZB, const u32* __restrict__ SBA,
                                                          const u32* __restrict__ BORD, Ctl* __restrict__ ctl,
                                                          const u32* __restrict__ A, const u32* __restrict__ B, double Nd,
                                                          u32* __restrict__ COLMAX, u64* __restrict__ RA11,
                                                          u32* __restrict__ RMAX, double* __restrict__ RF,
                                                          u64* __restrict__ RXL, int32_t* __restrict__ eci,
                                                          int32_t* __restrict__ ecj, int64_t* __restrict__ ecnt,
                                                          long long ecap, u32* __restrict__ wq) {
  __shared__ u32 s_key[CC_SLOTS];
  __shared__ u32 s_cnt[CC_SLOTS];
  __shared__ u32 s_hot[CB_ROWS];            // per row: the first detected label the class met in it
  __shared__ u32 s_hcnt[CB_ROWS * CC_SUB];  // its count, spread over CC_SUB counters
  __shared__ u64 r_a11[CB_ROWS], r_f[CB_ROWS], r_xlo[CB_ROWS], r_xhi[CB_ROWS];
  __shared__ u32 r_max[CB_ROWS], r_ai[CB_ROWS];
  __shared__ u32 s_item, s_over, s_sp, s_new, s_seen, s_est;
  __shared__ u32 s_stack[CC_STACK];  // pending classes: residue << 5 | log2 of the modulus
  const int tid = threadIdx.x;
  const u32 K = ctl->K;  // non-empty bands
  u32 q = blockIdx.x % WQ_QUEUES, left = WQ_QUEUES;  // thread 0's queue state (see wq_next)
  u64 nz = 0;
  for (;;) {
    if (tid == 0) s_item = wq_next(wq, K, q, left);
    __syncthreads();
    const u32 item = s_item;
    if (item == 0xFFFFFFFFu) break;
    const u32 band = BORD[item];
    const u32 base = SBS[band], len = SZB[band], a0 = SBA[band];
    const u32 rows = SBA[band + 1] - a0;
    for (u32 r = tid; r < rows; r += CC_THREADS) {
      r_a11[r] = 0;
      r_f[r] = 0;
      r_xlo[r] = 0;
      r_xhi[r] = 0;
      r_max[r] = 0;
      r_ai[r] = A[a0 + r];
    }
    if (tid == 0) {
      s_stack[0] = 0;  // residue 0 mod 1: the whole band
      s_sp = 1;
    }
    __syncthreads();
    while (s_sp > 0) {
      const u32 cls = s_stack[s_sp - 1];
      const u32 lg = cls & 31u, res = cls >> 5, mask = (1u << lg) - 1u;
      for (u32 i = tid; i < CC_SLOTS; i += CC_THREADS) {
        s_key[i] = EMPTY;
        s_cnt[i] = 0;
      }
      for (u32 r = tid; r < rows; r += CC_THREADS) s_hot[r] = EMPTY;
      for (u32 i = tid; i < rows * CC_SUB; i += CC_THREADS) s_hcnt[i] = 0;
      if (tid == 0) {
        s_over = 0;
        s_new = 0;
        s_seen = 0;
        s_est = len >> lg;  // the class's expected node count: a bound on its cells
      }
      __syncthreads();
      // each row's first detected label is taken from the band's first words, before the
      // counting threads would all meet it unset at once
      if ((u32)tid < len) {
        const u32 w = E[base + (u32)tid];
        const u32 b = w & 0xFFFFu;
        if (b != CMP_BAD_B && (b & mask) == res && s_hot[w >> 16] == EMPTY) atomicCAS(&s_hot[w >> 16], EMPTY, b);
      }
      __syncthreads();
      // a cell (row, detected label) is counted in the hash table, except the row's first
      // detected label met in this class, which is counted on the row's own counters
      // (in a band most nodes of a row share one detected label: one table slot would take
      // them all, and atomics on one address are performed one after another)
      u32 nnew = 0, nseen = 0;  // this thread's new table keys and counted words (first batch)
      auto insert = [&](u32 key, u32 c) {
        u32 h = hash_slot(key, CC_LOG2_SLOTS);
        for (u32 p = 0; p < CC_PROBE; ++p) {
          const u32 t = s_key[h];
          if (t == key) {
            atomicAdd(&s_cnt[h], c);
            return;
          }
          if (t == EMPTY) {
            if (lds_flag(&s_over)) return;  // the class is being split: stop adding keys
            const u32 old = atomicCAS(&s_key[h], EMPTY, key);
            if (old == EMPTY || old == key) {
              atomicAdd(&s_cnt[h], c);
              nnew += old == EMPTY;
              return;
            }
          }
          h = (h + 1u) & (CC_SLOTS - 1u);
        }
        s_over = 1;  // the table is too full for this class: split it
      };
      for (u32 e0 = 0; e0 < len; e0 += CC_THREADS * CC_BATCH) {
        u32 wv[CC_BATCH];  // a batch of the band's words, all loads in flight together
#pragma unroll
        for (int k = 0; k < CC_BATCH; ++k) {
          const u32 e = e0 + (u32)tid + (u32)k * CC_THREADS;
          wv[k] = e < len ? E[base + e] : 0xFFFFFFFFu;  // b = CMP_BAD_B: skipped
        }
#pragma unroll
        for (int k = 0; k < CC_BATCH; ++k) {
          const u32 w = wv[k];
          const u32 b = w & 0xFFFFu;
          if (b == CMP_BAD_B || (b & mask) != res) continue;
          ++nseen;
          const u32 r = w >> 16;
          u32 hb = s_hot[r];
          if (hb == EMPTY) {
            const u32 old = atomicCAS(&s_hot[r], EMPTY, b);
            hb = old == EMPTY ? b : old;
          }
          if (b == hb)
            atomicAdd(&s_hcnt[r * CC_SUB + ((u32)tid & (CC_SUB - 1))], 1u);
          else
            insert(w, 1u);
        }
        if (e0 == 0 && len > CC_THREADS * CC_BATCH) {
          // after the first batch: if new keys came at a rate that would overfill the table
          // before the class ends, split now (a nearly full table makes every probe long)
          const u64 a = wave_sum_u64(nnew), sn = wave_sum_u64(nseen);
          if ((tid & 63) == 0) {
            atomicAdd(&s_new, (u32)a);
            atomicAdd(&s_seen, (u32)sn);
          }
          __syncthreads();
          if (tid == 0 && s_seen > 0) {
            const u64 est = (u64)s_new * (u64)(len >> lg) / s_seen;
            if (est > CC_SLOTS * 5u / 8u) {
              s_est = (u32)est;
              s_over = 1;
            }
          }
          __syncthreads();
        }
        if (lds_flag(&s_over)) break;  // the class is being split
      }
      __syncthreads();
      if (!s_over) {
        for (u32 r = tid; r < rows; r += CC_THREADS) {
          const u32 hb = s_hot[r];
          if (hb == EMPTY) continue;
          u32 c = 0;
#pragma unroll
          for (int k = 0; k < CC_SUB; ++k) c += s_hcnt[r * CC_SUB + k];
          insert((r << 16) | hb, c);  // a new key: no entry with this label of the row went to the table
        }
      }
      __syncthreads();
      const bool over = s_over != 0;
      __syncthreads();  // every thread has read s_over before the stack changes
      if (over) {
        if (tid == 0) {
          // split to about 5,000 expected cells per class (the first batch's estimate, else
          // the class's node count), at least one and at most CC_JUMP levels further
          u32 want = lg + 1u;
          while (want < lg + CC_JUMP && want < 16u && (s_est >> (want - lg)) > CC_SLOTS * 5u / 8u) ++want;
          const u32 nchild = 1u << (want - lg);
          if (want > 16u || s_sp - 1u + nchild > (u32)CC_STACK) {
            atomicOr(&ctl->flags, F_STACK);  // never expected: 2^16 classes hold one label each
            s_sp = 0;
          } else {
            for (u32 c = 0; c < nchild; ++c) s_stack[s_sp - 1u + c] = ((res | (c << lg)) << 5) | want;
            s_sp = s_sp - 1u + nchild;
          }
        }
        __syncthreads();
        continue;
      }
      // visit every cell of the class once; a thread's slots are read, and their detected
      // labels' sizes loaded, before the first visit
      constexpr int VPT = 8;  // slots per thread and batch
      for (u32 i0 = 0; i0 < CC_SLOTS; i0 += CC_THREADS * VPT) {
      u32 vkey[VPT], vbj[VPT];
#pragma unroll
      for (int k = 0; k < VPT; ++k) vkey[k] = s_key[i0 + (u32)tid + (u32)k * CC_THREADS];
#pragma unroll
      for (int k = 0; k < VPT; ++k) vbj[k] = vkey[k] != EMPTY ? B[vkey[k] & 0xFFFFu] : 0u;
#pragma unroll
      for (int k = 0; k < VPT; ++k) {
        const u32 key = vkey[k];
        if (key == EMPTY) continue;
        const u32 x = s_cnt[i0 + (u32)tid + (u32)k * CC_THREADS];
        const u32 r = key >> 16, j = key & 0xFFFFu;
        const u32 bj = vbj[k];
        // row maxima: a plain read first, since most cells do not raise them
        if (x > r_max[r]) atomicMax(&r_max[r], x);
        const double f = 2.0 * (double)x / (double)((u64)r_ai[r] + (u64)bj);  // Eq. 3 ratio
        const u64 fb = (u64)__double_as_longlong(f);                           // f >= 0: the bits order as the values
        if (fb > r_f[r]) atomicMax(&r_f[r], fb);
        if (x > 1u) {  // a cell of one node adds nothing to C(n_ij, 2) or to S (log 1 = 0)
          atomicAdd(&r_a11[r], (u64)x * (u64)(x - 1u) / 2u);
          atomicMax(&COLMAX[j], x);
          // the cell's part of S, truncated to 2^-96 as the fixed-point sums do
          const double t = (double)x / Nd * log((double)x);
          const double x1 = t * 4294967296.0;
          const u64 l0 = (u64)x1;
          const double y1 = (x1 - (double)l0) * 4294967296.0;
          const u32 l1 = (u32)y1;
          const double z1 = (y1 - (double)l1) * 4294967296.0;
          const u32 l2 = (u32)z1;
          const u128 v = ((u128)l0 << 64) + ((u128)l1 << 32) + (u128)l2;
          const u64 lo = (u64)v;
          u64 hi = (u64)(v >> 64);
          const u64 old = atomicAdd(&r_xlo[r], lo);
          if (old + lo < old) hi += 1u;
          if (hi) atomicAdd(&r_xhi[r], hi);
        }
        nz += 1;
        if (ecap > 0) {
          const unsigned long long idx = atomicAdd(&ctl->export_count, 1ull);
          if ((long long)idx < ecap) {
            eci[idx] = (int32_t)(a0 + r);
            ecj[idx] = (int32_t)j;
            ecnt[idx] = (int64_t)x;
          }
        }
      }
      }
      __syncthreads();
      if (tid == 0) s_sp = s_sp - 1;
      __syncthreads();
    }
    for (u32 r = tid; r < rows; r += CC_THREADS) {
      const size_t i = (size_t)a0 + r;
      RA11[i] = r_a11[r];
      RMAX[i] = r_max[r];
      RF[i] = __longlong_as_double((long long)r_f[r]);
      RXL[2 * i] = r_xlo[r];
      RXL[2 * i + 1] = r_xhi[r];
    }
    __syncthreads();
  }
  nz = wave_sum_u64(nz);
  if ((tid & 63) == 0 && nz) atomicAdd(wq_sum(wq, blockIdx.x % WQ_QUEUES), (unsigned long long)nz);
}

}  // namespace cq
