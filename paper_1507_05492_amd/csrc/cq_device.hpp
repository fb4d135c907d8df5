// cq_device.hpp -- device-side building blocks shared by the gfx950 kernels:
// integer types, exact fixed-point accumulation, wave/block reductions and the
// per-workgroup LDS count tables (direct-indexed and open-addressing).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace cq {

typedef unsigned __int128 u128;
typedef uint64_t u64;
typedef uint32_t u32;

constexpr u32 SENT = 0xFFFFFFFFu;  // "no label" marker in staged label arrays
constexpr u32 EMPTY = 0xFFFFFFFFu; // empty hash slot

// device flag bits (cq_score_result.device_flags / cq_compare_result.device_flags)
constexpr u32 F_LABEL = 1u;   // a label outside [0, num_labels)
constexpr u32 F_GRAPH = 2u;   // malformed CSR (graph load only)
constexpr u32 F_EXPORT = 4u;  // export table too small
constexpr u32 F_STACK = 8u;   // internal: class stack exhausted (never expected)
constexpr u32 F_SEGMENT = 16u;  // internal: a community's entries exceed its segment (never expected)

// Control block at the start of every workspace.
struct Ctl {
  u32 flags;
  u32 K;          // non-empty communities (filled by the scan kernel)
  u32 kbig;       // groups whose segment holds at least GW_SPLIT entries (they come first in the order)
  u32 dense_rows;  // node pass of column-blocked graphs: buckets that wrote histogram rows
  unsigned long long export_count;
  unsigned long long reserved1;
  u32 changes;    // column-blocked node pass: label changes between consecutive stored ids
  u32 mode;       // column-blocked graphs: STAGE_BLOCKS or STAGE_ROWS, chosen from `changes`
  unsigned long long pad1[3];
};

// ---- work queues of the persistent per-community kernels ----------------------
// Atomics on one address are serialised where they are performed (about 12 ns each,
// measured on MI355X), so a single ticket counter caps a persistent kernel at one item
// per 12 ns however many workgroups wait.  The K items of an ordered list are therefore
// split into WQ_QUEUES interleaved queues (queue q hands out items q, q + 8, q + 16, ...,
// so each keeps the list's order), each with its counter on its own 128-byte line.  A
// workgroup starts on queue blockIdx.x % 8 (workgroups are dealt to the XCDs in turn)
// and moves on to the next queue when its own is empty, so none exits while work is left.
constexpr u32 WQ_QUEUES = 8;
constexpr u32 WQ_LINE = 32;                    // u32 words per counter line (128 bytes)
// tickets of the workgroup-per-group pass, per-queue 64-bit sums (cells), tickets of the
// wave-per-group pass
constexpr u32 WQ_WORDS = 3 * WQ_QUEUES * WQ_LINE;
constexpr size_t WQ_BYTES = 4 * (size_t)WQ_WORDS;
constexpr u32 WQ_WAVE = 2 * WQ_QUEUES * WQ_LINE;  // word offset of the wave pass's tickets

// Next item for the calling workgroup (thread 0 only), or 0xFFFFFFFF when every queue is
// empty.  q and left are thread 0's own state: start with q = blockIdx.x % 8, left = 8.
__device__ __forceinline__ u32 wq_next(u32* __restrict__ wq, u32 K, u32& q, u32& left) {
  while (left) {
    const u32 i = atomicAdd(&wq[q * WQ_LINE], 1u);
    const u64 item = (u64)q + (u64)WQ_QUEUES * i;
    if (item < K) return (u32)item;
    q = (q + 1u) % WQ_QUEUES;
    --left;
  }
  return 0xFFFFFFFFu;
}
// a 64-bit sum kept per queue on its own line (the second half of the region)
__device__ __forceinline__ unsigned long long* wq_sum(u32* wq, u32 q) {
  return reinterpret_cast<unsigned long long*>(wq + (WQ_QUEUES + q) * WQ_LINE);
}

// How a call on a column-blocked graph stages the neighbour labels (Ctl::mode; also
// reported in the result): through the column blocks with run claims, or through the
// graph's row-major copy with per-node offsets when the partition does not follow the
// stored order (short runs of equal labels make run claims as many as the nodes).
constexpr u32 STAGE_ROWS_ONLY = 0;  // the graph has no column blocks
constexpr u32 STAGE_BLOCKS = 1;
constexpr u32 STAGE_ROWS = 2;

// ---- exact fixed-point accumulation --------------------------------------
// A binary64 value t is turned into the integer round_toward_zero(t * 2^96) held in
// a 128-bit two's-complement word.  Integer addition is associative, so sums of
// such words are independent of the order in which terms arrive.  |t| < 2^31 is
// required; every term accumulated this way is bounded far below that.
__device__ __forceinline__ u128 fix96(double t) {
  double a = fabs(t);
  double f = ldexp(a, 96);
  u64 hi = __double2ull_rz(ldexp(f, -64));
  double rem = f - ldexp((double)hi, 64);  // exact: f and hi*2^64 share the leading bits
  u64 lo = __double2ull_rz(rem);
  u128 v = ((u128)hi << 64) | (u128)lo;
  return t < 0 ? (u128)(-(__int128)v) : v;
}
__device__ __forceinline__ double unfix96(u128 v) {
  bool neg = ((__int128)v) < 0;
  u128 a = neg ? (u128)(-(__int128)v) : v;
  double d = ldexp((double)(u64)(a >> 64), -32) + ldexp((double)(u64)a, -96);
  return neg ? -d : d;
}

// The same truncation, floor(t * 2^96), for terms known to lie in [0, 1), accumulated as
// three 32-bit limbs of the fraction in 64-bit words (fewer instructions than fix96).
struct Frac96Sum {
  u64 a = 0, b = 0, c = 0;
  __device__ __forceinline__ void add(double t) {
    const double x = t * 4294967296.0;  // 2^32
    const u32 l0 = (u32)x;               // truncation; each remainder below is exact
    const double y = (x - (double)l0) * 4294967296.0;
    const u32 l1 = (u32)y;
    const double z = (y - (double)l1) * 4294967296.0;
    const u32 l2 = (u32)z;
    a += l0;
    b += l1;
    c += l2;
  }
  // t in [0, 2^20): the integer part joins the first limb as well
  __device__ __forceinline__ void add_wide(double t) {
    const double x = t * 4294967296.0;
    const u64 l0 = (u64)x;
    const double y = (x - (double)l0) * 4294967296.0;
    const u32 l1 = (u32)y;
    const double z = (y - (double)l1) * 4294967296.0;
    const u32 l2 = (u32)z;
    a += l0;
    b += l1;
    c += l2;
  }
  __device__ __forceinline__ u128 value() const { return ((u128)a << 64) + ((u128)b << 32) + (u128)c; }
};

// 1/y for finite y >= 1: the hardware reciprocal estimate refined by two Newton-Raphson
// steps (r <- r + r(1 - yr), each squaring the relative error), which leaves it within
// about one unit in the last place; unlike a division it need not be correctly rounded.
__device__ __forceinline__ double recip_nr(double y) {
  double r = __builtin_amdgcn_rcp(y);
  double e = __builtin_fma(-y, r, 1.0);
  r = __builtin_fma(r, e, r);
  e = __builtin_fma(-y, r, 1.0);
  return __builtin_fma(r, e, r);
}

// ---- exact edge-weight sums --------------------------------------------------
// A float32 weight w in [2^-32, 2^32] is its 24-bit significand times 2^(e - 150), e the
// biased exponent (95 <= e <= 159), so w * 2^55 is the integer significand << (e - 95),
// below 2^88.  Sums of such integers are exact and independent of order, and 2^31 of
// them stay below 2^119.
constexpr float WEIGHT_MIN = 2.3283064365386963e-10f;  // 2^-32
constexpr float WEIGHT_MAX = 4294967296.0f;            // 2^32
constexpr u32 WEIGHT_EXP0 = 95;                        // biased exponent of 2^-32
__device__ __forceinline__ u128 fixw_f32(float w) {
  const u32 b = __float_as_uint(w);
  const u32 e = (b >> 23) & 0xFFu;
  return (u128)((b & 0x7FFFFFu) | 0x800000u) << (e - WEIGHT_EXP0);
}
// Exact sum of float32 weights in [WEIGHT_MIN, WEIGHT_MAX], times 2^55 (the value of
// fixw_f32), in two 64-bit words.  split() gives a weight's fixed-point value as
// (hi, lo): its 24-bit significand shifted left by s = biased exponent - WEIGHT_EXP0
// (0 <= s <= 64).
struct WeightSum {
  u64 lo = 0, hi = 0;
  static __device__ __forceinline__ void split(float w, u64& vlo, u64& vhi) {
    const u32 b = __float_as_uint(w);
    const u32 sh = ((b >> 23) & 0xFFu) - WEIGHT_EXP0;
    const u64 sig = (u64)((b & 0x7FFFFFu) | 0x800000u);
    vlo = sh < 64u ? sig << sh : 0ull;
    vhi = sh > 40u ? sig >> (64u - sh) : 0ull;
  }
  __device__ __forceinline__ void add(u64 vlo, u64 vhi) {
    lo += vlo;
    hi += vhi + (lo < vlo ? 1ull : 0ull);
  }
  __device__ __forceinline__ u128 value() const { return ((u128)hi << 64) | lo; }
};

// value / 2^55 of an exact weight sum
__device__ __forceinline__ double unfixw(u128 v) {
  return (double)(u64)(v >> 64) * 512.0 + (double)(u64)v * 2.7755575615628914e-17;  // 2^9, 2^-55
}

// ---- wave / block reductions (wave64) ---------------------------------------
__device__ __forceinline__ u64 wave_sum_u64(u64 x) {
  for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
  return x;
}
__device__ __forceinline__ u64 wave_max_u64(u64 x) {
  for (int o = 32; o > 0; o >>= 1) { u64 y = __shfl_xor(x, o, 64); x = y > x ? y : x; }
  return x;
}
__device__ __forceinline__ u32 wave_max_u32(u32 x) {
  for (int o = 32; o > 0; o >>= 1) { u32 y = __shfl_xor(x, o, 64); x = y > x ? y : x; }
  return x;
}
__device__ __forceinline__ double wave_max_f64(double x) {
  for (int o = 32; o > 0; o >>= 1) { double y = __shfl_xor(x, o, 64); x = y > x ? y : x; }
  return x;
}
__device__ __forceinline__ u128 wave_sum_u128(u128 x) {
  u64 lo = (u64)x, hi = (u64)(x >> 64);
  for (int o = 32; o > 0; o >>= 1) {
    u64 lo2 = __shfl_xor(lo, o, 64), hi2 = __shfl_xor(hi, o, 64);
    u64 s = lo + lo2;
    hi = hi + hi2 + (s < lo ? 1ull : 0ull);
    lo = s;
  }
  return ((u128)hi << 64) | lo;
}
// Deterministic double sum over a block: a fixed butterfly inside each wave, then
// wave totals combined in wave order by thread 0.  The result depends only on which
// thread held which value, never on timing.
template <int NW>
__device__ __forceinline__ double block_sum_f64(double x, double* sh) {
  for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
  int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) sh[w] = x;
  __syncthreads();
  double r = 0.0;
  if (threadIdx.x == 0) {
    for (int i = 0; i < NW; ++i) r += sh[i];
  }
  __syncthreads();
  return r;  // valid in thread 0
}

// inclusive scan of u32 inside a wave
__device__ __forceinline__ u32 wave_incl_scan(u32 x) {
  int lane = threadIdx.x & 63;
  for (int o = 1; o < 64; o <<= 1) {
    u32 y = __shfl_up(x, o, 64);
    if (lane >= o) x += y;
  }
  return x;
}

__device__ __forceinline__ u32 hash_slot(u32 key, u32 log2cap) {
  return (key * 0x9E3779B1u) >> (32 - log2cap);
}

}  // namespace cq
