// cq_lib.hip -- host runtime and C ABI (include/cq.h) of the gfx950 community-quality
// library: argument checks, workspace layout, launch sequencing on the caller's stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <chrono>
#include <condition_variable>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <thread>
#include <vector>

#include "cq.h"
#include "cq_kernels.hpp"
#include "cq_compare.hpp"
#include "srv_core.hpp"

using namespace cq;

struct cq_context {
  int device = 0;
  // column-blocked graphs: a partition whose labels change between at least this fraction
  // of consecutive stored nodes is staged through the graph's row-major copy
  double row_staging_from = 1.0 / 16.0;
  void* scratch = nullptr;  // device address of the library's scratch array on this device
  hipStream_t stream = nullptr;
  int num_cus = 256;
  void* pinned = nullptr;  // host staging for result structs (hipHostMalloc)
  u32* dscratch = nullptr; // 2 words used by graph checks
  char err[512] = {0};
  // stage timing
  uint32_t timing = 0;  // bit s: stage s is bracketed by events
  hipEvent_t ev[2 * CQ_MAX_STAGES] = {};
  bool recorded[CQ_MAX_STAGES] = {};
  double total_ms[CQ_MAX_STAGES] = {};
  int64_t counts[CQ_MAX_STAGES] = {};
};

struct cq_graph {
  cq_context* ctx = nullptr;
  int32_t n = 0;
  int64_t nnz = 0;
  const int32_t* rp = nullptr;    // CSR the kernels read (borrowed, or owned_rp)
  const int32_t* col = nullptr;
  const int32_t* perm = nullptr;  // graph row -> caller node id (null: identity)
  int64_t max_degree = 0;
  int64_t degree_bins[DEG_BINS] = {};  // rows per power-of-two degree bin (k_check_csr)
  uint32_t validated = 0;
  uint32_t reordered = 0;
  int32_t* owned_rp = nullptr;    // device memory owned by the handle (CQ_GRAPH_REORDER)
  int32_t* owned_col = nullptr;
  int32_t* owned_perm = nullptr;
  u32* rpb = nullptr;              // column blocks (owned; null when the graph is not blocked)
  int32_t* colb = nullptr;
  int32_t* rowb = nullptr;
  u32* deg_in = nullptr;           // label permutation plan (caller order -> stored order): degrees,
  u32* pos1 = nullptr;             // bucket slots and their stored ids; null when not built
  uint16_t* tgt = nullptr;         // offset of the slot's stored id in its bucket
  uint16_t* lrank = nullptr;       // column-blocked graphs: node numbers and slots of the plan's chunks
  u32* spos = nullptr;
  u32* pbstart = nullptr;          // first slot of every bucket (nb + 1)
  u32* sid = nullptr;              // graphs without column blocks: stored id of every caller node (k_perm_split)
  int perm_buckets = 0;
  const float* w = nullptr;        // edge weights in the stored entry order (borrowed or owned_w); null: unweighted
  float* owned_w = nullptr;
  float* wb = nullptr;             // weights in column-block order (with colb)
  double total_w = 0.0;            // W, summed exactly at load
  FarTable far{};                  // per block: entry ranges of the rows outside its span
  int64_t clusters = 0, largest_cluster = 0;  // of the locality order
  unsigned far_tiles = 0;          // most far-entry tiles of any block
  int64_t owned_bytes = 0;
  ~cq_graph() {
    if (owned_rp) (void)hipFree(owned_rp);
    if (owned_col) (void)hipFree(owned_col);
    if (owned_perm) (void)hipFree(owned_perm);
    if (rpb) (void)hipFree(rpb);
    if (colb) (void)hipFree(colb);
    if (rowb) (void)hipFree(rowb);
    for (u32* p : {deg_in, pos1, pbstart, sid})
      if (p) (void)hipFree(p);
    if (tgt) (void)hipFree(tgt);
    if (lrank) (void)hipFree(lrank);
    if (spos) (void)hipFree(spos);
    if (owned_w) (void)hipFree(owned_w);
    if (wb) (void)hipFree(wb);
  }
};

struct cq_batch_plan {
  cq_context* ctx = nullptr;
  uint32_t flags = 0;
  std::vector<cq_batch_task> tasks;
  std::vector<size_t> ws_off;  // per-task workspace offset
  size_t ws_total = 0;
  size_t items_off = 0;  // workspace offset of the flat (task, group) list of the group pass
  std::vector<std::array<int, 4>> groups;
  std::vector<int> group_np;
  int maxL = 1;
  int nsmall = 0;  // tasks with at most SMALL_L_MAX labels (the 128-thread group pass)
  // device tables (owned)
  void* d_tab = nullptr;
  size_t tab_bytes = 0;
  void* td = nullptr;  // cq::TaskDev[T]
  void* gd = nullptr;  // cq::GroupDev[ngroups]
  uint32_t *Wpre = nullptr, *Lpre = nullptr, *Gpre = nullptr, *Kpre = nullptr, *wq = nullptr;
  uint4* items = nullptr;  // ((task << 14) | group, segment start, length, 0) of every item of the group pass (workspace)
  uint32_t* RBpre[3] = {nullptr, nullptr, nullptr};  // per gather tile size: per XCD, tile prefixes over its groups
  uint32_t* XG[3] = {nullptr, nullptr, nullptr};     // per gather tile size: per XCD, its groups
  std::vector<size_t> il_off;  // per group: workspace offset of its interleaved labels
  uint32_t *XWpre = nullptr, *XT = nullptr;  // node pass: per XCD, its tasks' chunk prefix and (task, first chunk)
  uint32_t NXsum = 0;                        // node pass grid
  uint32_t Wsum = 0, Lsum = 0, Gsum = 0, RBsum[3] = {0, 0, 0};
  // binding
  void* ws = nullptr;
  cq_score_result* d_results = nullptr;
  bool bound = false;
  // tuning and replay
  int rsel = 1, occ = 1;
  double tuned_ms = 0.0;
  int from_cache = 0;
  int graph_nodes = 0;
  hipStream_t stream = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  hipEvent_t ev_in = nullptr, ev_out = nullptr;
  void* pinned = nullptr;
  ~cq_batch_plan() {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    if (d_tab) (void)hipFree(d_tab);
    if (ev_in) (void)hipEventDestroy(ev_in);
    if (ev_out) (void)hipEventDestroy(ev_out);
    if (stream) (void)hipStreamDestroy(stream);
    if (pinned) (void)hipHostFree(pinned);
  }
};

static_assert(sizeof(ScoreResultDev) == sizeof(cq_score_result), "score result layout");
static_assert(sizeof(CmpResultDev) == sizeof(cq_compare_result), "compare result layout");
static_assert(sizeof(PerComm) == sizeof(cq_per_community), "per-community layout");

namespace {

// ---- per-device scratch array (cq_score_partition_noalloc) ---------------------
// Device memory the library holds for callers that cannot allocate a workspace.  Each
// GPU the library is loaded on has its own copy, at its own address, until the process
// ends.  In host code `scratch` names a host-side stand-in, never the device memory:
// its address on a device comes from hipGetSymbolAddress, taken once per device when
// the first context on that device is created and kept in g_scratch_addr.
constexpr size_t SCRATCH_BYTES = (size_t)CQ_SCRATCH_BYTES;
constexpr int SCRATCH_DEVICES = 64;
__device__ __align__(256) unsigned char scratch[SCRATCH_BYTES];
std::mutex g_scratch_mu;
void* g_scratch_addr[SCRATCH_DEVICES] = {};

// Device address of the scratch array on `device` (which must be current), or null.
void* scratch_address(int device) {
  if (device < 0 || device >= SCRATCH_DEVICES) return nullptr;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_addr[device]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess) return nullptr;
    g_scratch_addr[device] = p;
  }
  return g_scratch_addr[device];
}

constexpr int64_t PRIV_MAX = 16384;    // labels one LDS-private node-histogram launch holds
constexpr int64_t RANGE_MAX = 8 * PRIV_MAX;  // labels counted in LDS-private launches, PRIV_MAX per range
constexpr int64_t DIRECT_MAX = 16384;  // labels handled by direct-indexed group tables
constexpr u32 HASH_WORDS = 32768;      // LDS words of the group hash table (16384 slots)
constexpr size_t ALIGN = 256;    // offsets of the arrays carved from a workspace
constexpr size_t WS_ALIGN = 16;  // workspaces: the kernels load 16-byte vectors from the arrays

enum Stage { ST_SETUP = 0, ST_NODE, ST_COLSCAN, ST_ORDER, ST_GATHER, ST_GROUPS, ST_FINAL, ST_HIST_B, ST_SCATTER, ST_COUNT };
const char* const kStageNames[ST_COUNT] = {"setup", "node_pass", "column_scan", "scan_order", "edge_gather",
                                           "group_count", "final_reduce", "label_hist_b", "node_scatter"};
static_assert(ST_COUNT <= CQ_MAX_STAGES, "stage ids");

// Brackets one stage with events when timing is on (synchronous calls only).
struct StageMark {
  cq_context* ctx;
  int st;
  bool on;
  StageMark(cq_context* c, int s, bool timed) : ctx(c), st(s), on(timed && ((c->timing >> s) & 1u)) {
    if (on) (void)hipEventRecord(ctx->ev[2 * st], ctx->stream);
  }
  ~StageMark() {
    if (on) {
      (void)hipEventRecord(ctx->ev[2 * st + 1], ctx->stream);
      ctx->recorded[st] = true;
    }
  }
};

void collect_stage_times(cq_context* ctx) {
  for (int i = 0; i < ST_COUNT; ++i) {
    if (!ctx->recorded[i]) continue;
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, ctx->ev[2 * i], ctx->ev[2 * i + 1]) == hipSuccess) {
      ctx->total_ms[i] += ms;
      ctx->counts[i] += 1;
    }
    ctx->recorded[i] = false;
  }
}

cq_status fail(cq_context* ctx, cq_status s, const char* fmt, ...) {
  if (ctx) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(ctx->err, sizeof(ctx->err), fmt, ap);
    va_end(ap);
  }
  return s;
}

struct Carve {
  size_t off = 0;
  size_t take(size_t bytes) {
    size_t o = off;
    off += (std::max<size_t>(bytes, 1) + ALIGN - 1) & ~(ALIGN - 1);
    return o;
  }
};

// Nodes per workgroup of the private-histogram node passes: about 256 workgroups, at
// most max_chunk nodes each.
int pick_chunk(int64_t n, int64_t max_chunk = 65536, int64_t min_chunk = 1024) {
  int64_t c = min_chunk;
  while (c < max_chunk && c * 256 < n) c <<= 1;
  return (int)c;
}
// Node chunk limit when the labels span several LDS ranges (the histogram rows are W x L).
constexpr int64_t RANGE_CHUNK_MAX = 1 << 18;
// Workgroups of a scoring node pass over several label ranges: the CUs of the GPU
constexpr int64_t RANGE_WGS = 256;
// The caller-order node pass of column-blocked graphs (k_node_perm) is bound by its
// scattered label stores and gains from more, smaller workgroups; its column scan only
// needs totals, so the extra histogram rows cost little.
constexpr int64_t PERM_CHUNK_MAX = 16384;

unsigned grid_for(int64_t items, int per_block, unsigned cap) {
  int64_t g = (items + per_block - 1) / per_block;
  return (unsigned)std::max<int64_t>(1, std::min<int64_t>(g, cap));
}

unsigned colscan_grid(int64_t L) { return grid_for(L, CS_LABELS, 1u << 30); }

struct ScoreLayout {
  bool priv, small;  // small: labels fit 16 bits (num_labels <= 65535)
  int chunk, W, G;
  size_t ctl, wq, N, D, start, order, I, NP, PEN, SZ, cursor, loc, HN, HD, RL, labx, CB, parts, res, total;
  size_t CW, SW, IW, PENW, INVN;  // weighted graphs only (0 otherwise)
};

ScoreLayout score_layout(int64_t n, int64_t nnz, int64_t L, bool weighted = false, int64_t max_chunk = 65536,
                         int64_t min_chunk = 1024) {
  ScoreLayout s{};
  Carve c;
  s.priv = L <= RANGE_MAX;
  s.small = L <= 65535;
  const size_t lt = s.small ? 2 : 4;
  // several label ranges: fewer, larger node chunks keep the W x L histogram rows small
  // several label ranges: one workgroup per CU holds a range's LDS histograms, so the
  // nodes are cut into at most RANGE_WGS chunks (one wave of workgroups, no tail)
  s.chunk = L > PRIV_MAX ? (int)std::max<int64_t>(1024, ((n + RANGE_WGS - 1) / RANGE_WGS + 1023) / 1024 * 1024)
                         : pick_chunk(n, std::max(max_chunk, min_chunk), min_chunk);
  s.W = (int)((n + s.chunk - 1) / s.chunk);
  s.G = (int)std::min<int64_t>(128, std::max<int64_t>(1, (L + 1023) / 1024));
  s.ctl = c.take(sizeof(Ctl));
  s.wq = c.take(WQ_BYTES);
  s.N = c.take(4 * L);
  s.D = c.take(4 * L);
  s.start = c.take(4 * L);
  s.order = c.take(4 * L);
  s.I = c.take(4 * L);
  s.NP = c.take(4 * L);
  s.PEN = c.take(16 * L);
  s.SZ = s.priv ? 0 : c.take(8 * L);
  s.cursor = c.take(8 * L);  // u32 run cursors, or u64 (cursor, own-label count) with compact staging
  s.loc = c.take(4 * n);
  s.HN = s.priv ? c.take(4 * (size_t)s.W * L) : 0;
  s.HD = s.priv ? c.take(4 * (size_t)s.W * L) : 0;
  s.RL = c.take(4 * (size_t)(((n + (1 << PERM_SHIFT) - 1) >> PERM_SHIFT) + 1));  // dense-bucket rows of the node pass
  s.labx = c.take(lt * n);
  s.CB = c.take(lt * nnz);
  s.parts = c.take(std::max(sizeof(ScorePart), sizeof(WScorePart)) * s.G);
  s.res = c.take(sizeof(ScoreResultDev));
  if (weighted) {
    s.CW = c.take(4 * (size_t)nnz);
    s.SW = c.take(16 * (size_t)L);
    s.IW = c.take(16 * (size_t)L);
    s.PENW = c.take(16 * (size_t)L);
    s.INVN = c.take(8 * (size_t)L);
  }
  s.total = c.off;
  return s;
}

// A batched task's layout: a batch has parallelism across its tasks, so its node pass
// takes chunks of at least 4,096 nodes (4 per thread), which keeps the per-workgroup
// histogram rows (W x L per task) few.  Never larger than the single-call layout.
ScoreLayout batch_task_layout(int64_t n, int64_t nnz, int64_t L) { return score_layout(n, nnz, L, false, 65536, 4096); }

// The layout of one scoring call on graph g (the node pass it takes decides the chunk).
ScoreLayout graph_score_layout(const cq_graph* g, int64_t L) {
  const bool perm = g->rpb && g->pos1 && L <= PRIV_MAX;
  return score_layout(g->n, g->nnz, L, g->w != nullptr, perm ? PERM_CHUNK_MAX : 65536);
}

struct CmpLayout {
  bool privA, privB, small;  // small: detected labels fit 16 bits
  bool bands;                // both label spaces fit 16 bits: the band path (cq_compare.hpp)
  int chunk, W, Wb, Ga, Gb;
  int Wa, rounds, Wc, nbmax;  // band path: histogram grid of A, rounds per chunk, chunks, bands at most
  u32 T;                      // band path: nodes per band aimed at
  size_t ctl, wq, A, B, start, order, COLMAX, RA11, RMAX, RF, RXL, SZ, loc, HN, HB, CB, parts, res, total;
  size_t HA, sbk, SBA, SZB, SBS, CUR, BORD, E;
};

// Band path sizes: bands of about T nodes, at least 8,192 (a band's cells then mostly fit
// the cell table in one class) and at most about 1,024 bands by size (every chunk claims
// one run per band it has nodes of); chunks of whole rounds of CP_CHUNK nodes, at most
// about 1,024 chunks.
constexpr int64_t CB_MIN_T = 8192;
constexpr int64_t CB_MAX_BANDS_BY_SIZE = 1024;
constexpr int64_t CP_MAX_CHUNKS = 1024;

CmpLayout cmp_layout(int64_t n, int64_t La, int64_t Lb) {
  CmpLayout s{};
  Carve c;
  s.privA = La <= RANGE_MAX;
  s.privB = Lb <= RANGE_MAX;
  s.small = Lb <= 65535;
  s.bands = La <= 65535 && Lb <= 65535;
  s.Wb = (int)std::min<int64_t>(256, std::max<int64_t>(1, (n + 8191) / 8192));
  s.Ga = (int)std::min<int64_t>(64, std::max<int64_t>(1, (La + 1023) / 1024));
  s.Gb = (int)std::min<int64_t>(64, std::max<int64_t>(1, (Lb + 1023) / 1024));
  if (s.bands) {
    s.Wa = s.Wb;
    s.T = (u32)std::max<int64_t>(CB_MIN_T, (n + CB_MAX_BANDS_BY_SIZE - 1) / CB_MAX_BANDS_BY_SIZE);
    s.nbmax = (int)(n / s.T + (La + CB_ROWS - 1) / CB_ROWS + 2);
    s.rounds = (int)std::max<int64_t>(1, (n + CP_CHUNK * CP_MAX_CHUNKS - 1) / (CP_CHUNK * CP_MAX_CHUNKS));
    s.Wc = (int)((n + (int64_t)CP_CHUNK * s.rounds - 1) / ((int64_t)CP_CHUNK * s.rounds));
    s.ctl = c.take(sizeof(Ctl));
    s.wq = c.take(WQ_BYTES);
    s.A = c.take(4 * La);
    s.B = c.take(4 * Lb);
    s.COLMAX = c.take(4 * Lb);
    s.RA11 = c.take(8 * La);
    s.RMAX = c.take(4 * La);
    s.RF = c.take(8 * La);
    s.RXL = c.take(16 * La);
    s.HA = c.take(4 * (size_t)s.Wa * La);
    s.HB = c.take(4 * (size_t)s.Wb * Lb);
    s.sbk = c.take(4 * La);
    s.SBA = c.take(4 * ((size_t)s.nbmax + 1));
    s.SZB = c.take(4 * (size_t)s.nbmax);
    s.SBS = c.take(4 * ((size_t)s.nbmax + 1));
    s.CUR = c.take(4 * (size_t)s.nbmax);
    s.BORD = c.take(4 * (size_t)s.nbmax);
    s.E = c.take(4 * (size_t)n);
    s.parts = c.take(sizeof(CmpPart) * (s.Ga + s.Gb));
    s.res = c.take(sizeof(CmpResultDev));
    s.total = c.off;
    return s;
  }
  s.chunk = pick_chunk(n, La > PRIV_MAX ? RANGE_CHUNK_MAX : 65536);
  s.W = (int)((n + s.chunk - 1) / s.chunk);
  s.ctl = c.take(sizeof(Ctl));
  s.wq = c.take(WQ_BYTES);
  s.A = c.take(4 * La);
  s.B = c.take(4 * Lb);
  s.start = c.take(4 * La);
  s.order = c.take(4 * La);
  s.COLMAX = c.take(4 * Lb);
  s.RA11 = c.take(8 * La);
  s.RMAX = c.take(4 * La);
  s.RF = c.take(8 * La);
  s.RXL = c.take(16 * La);
  s.SZ = s.privA ? 0 : c.take(8 * La);
  s.loc = c.take(4 * n);
  s.HN = s.privA ? c.take(4 * (size_t)s.W * La) : 0;
  s.HB = s.privB ? c.take(4 * (size_t)s.Wb * Lb) : 0;
  s.CB = c.take((s.small ? 2 : 4) * n);
  s.parts = c.take(sizeof(CmpPart) * (s.Ga + s.Gb));
  s.res = c.take(sizeof(CmpResultDev));
  s.total = c.off;
  return s;
}

template <class T>
T* at(void* ws, size_t off) {
  return reinterpret_cast<T*>(static_cast<char*>(ws) + off);
}

cq_status launch_status(cq_context* ctx, const char* what) {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(ctx, CQ_E_DEVICE, "%s: %s", what, hipGetErrorString(e));
  return CQ_OK;
}

void fill(u32* p, size_t words, u32 v, hipStream_t s) {
  k_fill_u32<<<grid_for((int64_t)words, 256, 1024), 256, 0, s>>>(p, words, v);
}

template <class V, class LT, int NT = GBLOCK>
unsigned group_grid(cq_context* ctx, size_t lds_bytes) {
  int nb = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_groups<V, LT, NT>, NT, lds_bytes) != hipSuccess || nb < 1) nb = 1;
  return (unsigned)(ctx->num_cus * nb);
}

cq_status map_flags(cq_context* ctx, u32 flags) {
  if (flags & F_LABEL) return fail(ctx, CQ_E_LABEL_RANGE, "a label is outside [0, num_labels)");
  if (flags & F_STACK) return fail(ctx, CQ_E_DEVICE, "internal: group table split limit reached");
  if (flags & F_SEGMENT) return fail(ctx, CQ_E_DEVICE, "internal: segment overflow in the edge pass");
  if (flags & F_EXPORT) return fail(ctx, CQ_E_CAPACITY, "export table capacity too small");
  return CQ_OK;
}

// Moves the caller's labels to the stored node order: labx[stored id] = label, or the
// sentinel (flagged) when out of range.  tmp holds n labels and may alias the per-node
// offsets, which are written only afterwards.  scratch (scratch_bytes) is free workspace
// (the staged-entry array, written only by the edge pass): with the graph's stored ids
// and room for 8 bytes per node, the move takes the two streaming passes of
// k_perm_split / k_perm_place; otherwise the bucket plan's scatter and per-bucket pass.
template <class LT>
void stage_labels(const cq_graph* g, const int32_t* labels, int32_t L, LT* tmp, LT* labx, Ctl* ctl, void* scratch,
                  size_t scratch_bytes, hipStream_t s) {
  const int n = g->n;
  const int nsb = (int)(((int64_t)n + SB_MASK) >> SB_SHIFT);
  const size_t stage_bytes = 8 * ((size_t)nsb << SB_SHIFT);
  if (g->sid && nsb <= SB_MAX && stage_bytes + 4 * (size_t)SB_MAX <= scratch_bytes) {
    auto* stage = static_cast<unsigned long long*>(scratch);
    u32* gcur = reinterpret_cast<u32*>(static_cast<char*>(scratch) + stage_bytes);
    fill(gcur, (size_t)nsb, 0, s);
    k_perm_split<LT><<<(unsigned)(((int64_t)n + PS_NODES - 1) / PS_NODES), 1024, 0, s>>>(n, labels, g->sid, L, nsb, gcur,
                                                                                        stage, ctl);
    const unsigned groups = (unsigned)((nsb + 7) / 8);
    k_perm_place<LT><<<8u * PP_PARTS * groups, 1024, 0, s>>>(n, nsb, stage, labx);
    return;
  }
  k_perm_scatter<LT><<<grid_for(n, 256 * 8, 8192), 256, 0, s>>>(n, labels, g->pos1, L, tmp, ctl);
  k_perm_apply<LT><<<g->perm_buckets, 1024, ((size_t)1 << PERM_SHIFT) * sizeof(LT), s>>>(n, g->pbstart, g->tgt, tmp, labx);
}

// The scoring path with staged labels of type LT (u16 when num_labels <= 65535).
template <class LT>
void score_launch(cq_context* ctx, const cq_graph* g, const int32_t* labels, int32_t L, void* ws, const ScoreLayout& lay,
                  ScoreResultDev* d_out, const cq_per_community* per_comm, const cq_pair_table* pairs, bool timed) {
  const int64_t n = g->n, nnz = g->nnz;
  hipStream_t s = ctx->stream;
  Ctl* ctl = at<Ctl>(ws, lay.ctl);
  u32* N = at<u32>(ws, lay.N);
  u32* D = at<u32>(ws, lay.D);
  u32* start = at<u32>(ws, lay.start);
  u32* order = at<u32>(ws, lay.order);
  u32* I = at<u32>(ws, lay.I);
  u32* NP = at<u32>(ws, lay.NP);
  u64* PEN = at<u64>(ws, lay.PEN);
  u32* loc = at<u32>(ws, lay.loc);
  LT* labx = at<LT>(ws, lay.labx);
  LT* CB = at<LT>(ws, lay.CB);
  float* CW = g->w ? at<float>(ws, lay.CW) : nullptr;  // weights staged beside the labels
  ScorePart* parts = at<ScorePart>(ws, lay.parts);
  const u32* PM = nullptr;
  bool dual_rows = false;  // column-blocked graph whose staging is chosen on the device
  {
    StageMark mk(ctx, ST_SETUP, timed);
    // the control block and the work queues in one launch
    k_cmp_clear<<<grid_for((int64_t)(sizeof(Ctl) / 4) + WQ_WORDS, 256, 64), 256, 0, s>>>(
        reinterpret_cast<u32*>(ctl), (int)(sizeof(Ctl) / 4), at<u32>(ws, lay.wq), nullptr, 0);
    if (!lay.priv) fill(at<u32>(ws, lay.SZ), 2 * (size_t)L, 0, s);
    // run cursors of column-blocked graphs: cleared by the column scan on the
    // private-histogram path, here otherwise
    if (g->rpb && !(L <= PRIV_MAX && g->pos1)) fill(at<u32>(ws, lay.cursor), 2 * (size_t)L, 0, s);
    // weighted column-blocked graphs: the edge pass adds each community's own-label weights here
    if (CW && g->rpb) fill(at<u32>(ws, lay.IW), 4 * (size_t)L, 0, s);
  }
  if (L <= PRIV_MAX && g->rpb && g->pos1) {
    // column-blocked graph: move the labels with the bucket plan and count per label (the
    // blocked edge pass needs no per-node offsets)
    u32* HN = at<u32>(ws, lay.HN);
    u32* HD = at<u32>(ws, lay.HD);
    LT* tmp = reinterpret_cast<LT*>(loc);  // per-node offsets are not used on this path
    if (sizeof(LT) == 2 && L <= APPLY_COUNT_MAX_L && g->lrank) {
      // count in the stored order while moving the labels there (labels come in runs)
      u32* rows = at<u32>(ws, lay.RL);
      {
        StageMark mk(ctx, ST_NODE, timed);
        const unsigned gs = (unsigned)(((int64_t)n + PERM_NODES - 1) / PERM_NODES);  // the plan's chunks
        k_node_scatter<LT><<<gs, 1024, 0, s>>>((int)n, labels, g->lrank, g->spos, L, tmp, N, D, ctl);
        k_perm_apply_count<<<g->perm_buckets, 1024, ((size_t)1 << PERM_SHIFT) * 2 + 8 * (size_t)L, s>>>(
            g->pbstart, g->tgt, reinterpret_cast<const uint16_t*>(tmp), reinterpret_cast<uint16_t*>(labx), g->rp, L, N, D, HN, HD,
            rows, ctl);
      }
      // A partition out of the stored order (many label changes along it) would make the
      // column blocks' run claims as many as the nodes: k_colscan_rows then picks staging
      // through the row-major copy, whose per-node offsets come from the gated launches
      // below (they return at once when the blocks are kept).
      const bool dual = !CW;
      {
        StageMark mk(ctx, ST_COLSCAN, timed);
        const double f = ctx->row_staging_from;
        const u32 rows_from = !dual ? 0xFFFFFFFFu : f <= 0.0 ? 0u : (f >= 1.0 ? 0xFFFFFFFFu : (u32)std::ceil(f * (double)n));
        k_colscan_rows<<<grid_for(L, 256, 1u << 30), 256, 0, s>>>(L, HN, HD, rows, ctl, N, D,
                                                                  at<unsigned long long>(ws, lay.cursor), rows_from);
        if (dual) {
          // after k_colscan_rows: it set the mode and has read the dense buckets' rows of HN/HD
          k_node_priv<true, LT, true><<<lay.W, 1024, 2 * (size_t)L * 4, s>>>((int)n, labels, g->perm, g->rp, L, lay.chunk, HN,
                                                                           HD, loc, labx, ctl, 0, L, STAGE_ROWS);
          k_colscan<true, true><<<colscan_grid(L), CS_LABELS * CS_GROUPS, 0, s>>>(lay.W, L, HN, HD, N, D, nullptr, ctl,
                                                                             STAGE_ROWS);
        }
        dual_rows = dual;
      }
    } else {
      // more labels than LDS holds beside a bucket: count in the caller's order
      {
        StageMark mk(ctx, ST_NODE, timed);
        k_node_perm<LT><<<lay.W, 1024, 2 * (size_t)L * 4, s>>>((int)n, labels, g->deg_in, g->pos1, L, lay.chunk, HN, HD, tmp,
                                                               ctl);
        k_perm_apply<LT><<<g->perm_buckets, 1024, ((size_t)1 << PERM_SHIFT) * sizeof(LT), s>>>((int)n, g->pbstart, g->tgt, tmp,
                                                                                            labx);
      }
      {
        StageMark mk(ctx, ST_COLSCAN, timed);
        k_colscan<true, false><<<colscan_grid(L), CS_LABELS * CS_GROUPS, 0, s>>>(lay.W, L, HN, HD, N, D,
                                                                            at<unsigned long long>(ws, lay.cursor));
      }
    }
    PM = HD;
  } else if (lay.priv) {
    u32* HN = at<u32>(ws, lay.HN);
    u32* HD = at<u32>(ws, lay.HD);
    {
      StageMark mk(ctx, ST_NODE, timed);
      // move the labels to the stored order first (streaming), then count in that order;
      // without a plan the first range's launch reads them and writes labx
      if (g->pos1)
        stage_labels<LT>(g, labels, L, reinterpret_cast<LT*>(loc), labx, ctl, CB, sizeof(LT) * (size_t)nnz, s);
      for (int64_t lb = 0; lb < L; lb += PRIV_MAX) {
        const int lr = (int)std::min<int64_t>(PRIV_MAX, L - lb);
        const size_t shm = 2 * (size_t)lr * 4;
        if (g->pos1 || lb > 0)
          k_node_priv<true, LT, true><<<lay.W, 1024, shm, s>>>((int)n, labels, g->perm, g->rp, L, lay.chunk, HN, HD, loc, labx,
                                                             ctl, (int)lb, lr);
        else
          k_node_priv<true, LT><<<lay.W, 1024, shm, s>>>((int)n, labels, g->perm, g->rp, L, lay.chunk, HN, HD, loc, labx, ctl, 0,
                                                         lr);
      }
    }
    {
      StageMark mk(ctx, ST_COLSCAN, timed);
      k_colscan<true, true><<<colscan_grid(L), CS_LABELS * CS_GROUPS, 0, s>>>(lay.W, L, HN, HD, N, D);
    }
    PM = HD;
  } else {
    unsigned long long* SZ = at<unsigned long long>(ws, lay.SZ);
    {
      StageMark mk(ctx, ST_NODE, timed);
      if (g->pos1) {
        stage_labels<LT>(g, labels, L, reinterpret_cast<LT*>(loc), labx, ctl, CB, sizeof(LT) * (size_t)nnz, s);
        k_node_global<true, LT, true><<<grid_for(n, 256, 8192), 256, 0, s>>>((int)n, labels, g->perm, g->rp, L, SZ, loc, labx,
                                                                            ctl);
      } else {
        k_node_global<true, LT><<<grid_for(n, 256, 8192), 256, 0, s>>>((int)n, labels, g->perm, g->rp, L, SZ, loc, labx, ctl);
      }
    }
    {
      StageMark mk(ctx, ST_COLSCAN, timed);
      k_unpack<<<grid_for(L, 256, 4096), 256, 0, s>>>(L, SZ, N, D);
    }
  }
  {
    StageMark mk(ctx, ST_ORDER, timed);
    k_scan_order<<<1, 1024, 0, s>>>(L, N, D, start, order, ctl);
  }
  {
    StageMark mk(ctx, ST_GATHER, timed);
    if (g->rpb) {
      const int64_t span = (n + COL_BLOCKS - 1) / COL_BLOCKS;
      const unsigned own_groups = (unsigned)((span + BT_ROWS - 1) / BT_ROWS);
      const unsigned grid = COL_BLOCKS * (own_groups + g->far_tiles);
      if (CW)
        k_gather_blocked<LT, true><<<grid, BT_THREADS, 0, s>>>((int)n, (int)span, g->rpb, g->colb, g->rowb, g->far, own_groups,
                                                               g->far_tiles, labx, start, D, at<u32>(ws, lay.cursor), ctl, CB,
                                                               g->wb, CW, at<unsigned long long>(ws, lay.IW));
      else
        k_gather_blocked<LT, false><<<grid, BT_THREADS, 0, s>>>((int)n, (int)span, g->rpb, g->colb, g->rowb, g->far, own_groups,
                                                                g->far_tiles, labx, start, D, at<u32>(ws, lay.cursor), ctl, CB,
                                                                nullptr, nullptr, nullptr);
      if (dual_rows) {
        // the other choice: every entry staged at its row's offset, through the row-major copy
        const unsigned gr = std::min(grid_for(n, GROWS, 1u << 30), (unsigned)(ctx->num_cus * 64));
        k_gather<true, LT, false><<<gr, GROWS, 0, s>>>((int)n, g->rp, g->col, labx, L, lay.chunk, PM, start, loc, CB, nullptr,
                                                       nullptr, ctl);
      }
    } else {
      const unsigned grid = 8u * (unsigned)((((int64_t)n + GROWS - 1) / GROWS + 7) / 8);  // one workgroup per tile
      if (lay.priv && CW)
        k_gather<true, LT, true><<<grid, GROWS, 0, s>>>((int)n, g->rp, g->col, labx, L, lay.chunk, PM, start, loc, CB, g->w, CW);
      else if (lay.priv)
        k_gather<true, LT, false><<<grid, GROWS, 0, s>>>((int)n, g->rp, g->col, labx, L, lay.chunk, PM, start, loc, CB, nullptr,
                                                        nullptr);
      else if (CW)
        k_gather<false, LT, true><<<grid, GROWS, 0, s>>>((int)n, g->rp, g->col, labx, L, lay.chunk, PM, start, loc, CB, g->w, CW);
      else
        k_gather<false, LT, false><<<grid, GROWS, 0, s>>>((int)n, g->rp, g->col, labx, L, lay.chunk, PM, start, loc, CB, nullptr,
                                                         nullptr);
    }
  }
  ScoreVis vis;
  vis.N = N;
  vis.twom = (double)nnz;
  vis.I = I;
  vis.NP = NP;
  vis.PEN = PEN;
  vis.eci = pairs ? pairs->ci : nullptr;
  vis.ecj = pairs ? pairs->cj : nullptr;
  vis.ecnt = pairs ? pairs->count : nullptr;
  vis.ecap = pairs ? pairs->capacity : 0;
  vis.ctl = ctl;
  const u32 lds_words = L <= DIRECT_MAX ? std::max<u32>(((u32)L + 3u) & ~3u, 128u) : HASH_WORDS;
  const size_t lds = (size_t)lds_words * 4;
  PerComm pc;
  std::memset(&pc, 0, sizeof(pc));
  if (per_comm) std::memcpy(&pc, per_comm, sizeof(pc));
  if (CW) {
    // weighted graph: direct tables only (L <= HASH_WORDS was checked by the caller)
    WeightedOut wo;
    wo.SW = at<u64>(ws, lay.SW);
    wo.IW = at<u64>(ws, lay.IW);
    wo.PENW = at<u64>(ws, lay.PENW);
    double* invN = at<double>(ws, lay.INVN);
    wo.invN = invN;
    wo.twoW = 2.0 * g->total_w;
    {
      StageMark mk(ctx, ST_GROUPS, timed);
      k_inv_sizes<<<grid_for(L, 256, 1024), 256, 0, s>>>(L, N, invN);
      int nb = 0;
      if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_groups_w<LT>, GBLOCK, lds) != hipSuccess || nb < 1) nb = 1;
      // column-blocked graphs stage compactly: lengths and own-label counts in the cursors
      const unsigned long long* cur64 = g->rpb ? at<unsigned long long>(ws, lay.cursor) : nullptr;
      k_groups_w<LT><<<(unsigned)(ctx->num_cus * nb), GBLOCK, lds, s>>>(CB, CW, start, D, order, ctl, (u32)L, vis, wo,
                                                                        cur64, at<u32>(ws, lay.wq));
    }
    WScorePart* wparts = reinterpret_cast<WScorePart*>(parts);
    {
      StageMark mk(ctx, ST_FINAL, timed);
      k_score_final1_w<<<lay.G, FBLOCK, 0, s>>>(L, N, D, I, NP, wo.SW, wo.IW, wo.PENW, g->total_w, pc, wparts);
      k_score_final2_w<<<1, 64, 0, s>>>(lay.G, wparts, n, nnz, g->total_w, vis.ecap, ctl, d_out, g->rpb ? 1u : 0u);
    }
    return;
  }
  {
    StageMark mk(ctx, ST_GROUPS, timed);
    // column-blocked graphs stage compactly (see k_gather_blocked): lengths and own-label counts in the cursors
    const unsigned long long* cur64 = g->rpb ? at<unsigned long long>(ws, lay.cursor) : nullptr;
    // Label spaces beyond the direct LDS table (16-bit labels): groups of degree sum below
    // GW_SPLIT are counted one per wave after the workgroup-per-group pass has taken the
    // others.  The choice depends on num_labels and the degree sums only, so a group takes
    // the same pass in every storage; batches (num_labels <= 16384) never split.  With
    // direct tables the split costs more than it gains: the large groups' tail no longer
    // overlaps the small ones.
    // Direct tables (the batch's label spaces too) take workgroups of GBLOCK_SMALL
    // threads up to SMALL_L_MAX labels and GBLOCK_DIRECT beyond, larger label spaces
    // GBLOCK_WIDE; a label count always takes the same size, so a task scores the same
    // bits alone and in a batch (each thread sums its own visits).
    const bool waves = sizeof(LT) == 2 && L > DIRECT_MAX;
    // (no more persistent workgroups than communities can be: a small graph's call would
    // otherwise launch thousands that find the queues empty)
    const unsigned lcap = (unsigned)std::max<int64_t>(1, L);
    if (L <= (int32_t)SMALL_L_MAX)
      k_groups<ScoreVis, LT, GBLOCK_SMALL><<<std::min(group_grid<ScoreVis, LT, GBLOCK_SMALL>(ctx, lds), lcap), GBLOCK_SMALL,
                                             lds, s>>>(CB, start, D, order, ctl, (u32)L, lds_words, vis, cur64,
                                                       at<u32>(ws, lay.wq), false);
    else if (L <= DIRECT_MAX)
      k_groups<ScoreVis, LT, GBLOCK_DIRECT><<<std::min(group_grid<ScoreVis, LT, GBLOCK_DIRECT>(ctx, lds), lcap), GBLOCK_DIRECT,
                                              lds, s>>>(CB, start, D, order, ctl, (u32)L, lds_words, vis, cur64,
                                                        at<u32>(ws, lay.wq), false);
    else
      k_groups<ScoreVis, LT, GBLOCK_WIDE><<<group_grid<ScoreVis, LT, GBLOCK_WIDE>(ctx, lds), GBLOCK_WIDE, lds, s>>>(
          CB, start, D, order, ctl, (u32)L, lds_words, vis, cur64, at<u32>(ws, lay.wq), waves);
    if (waves) {
      int nb = 0;
      if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_groups_wave<ScoreVis>, 64 * GW_WAVES, 0) != hipSuccess || nb < 1)
        nb = 1;
      k_groups_wave<ScoreVis><<<(unsigned)(ctx->num_cus * nb), 64 * GW_WAVES, 0, s>>>(
          reinterpret_cast<const uint16_t*>(CB), start, D, order, ctl, (u32)L, vis, at<u32>(ws, lay.wq), cur64);
    }
  }
  {
    StageMark mk(ctx, ST_FINAL, timed);
    k_score_final1<<<lay.G, FBLOCK, 0, s>>>(L, N, D, I, NP, PEN, (double)nnz, pc, parts);
    k_score_final2<<<1, 64, 0, s>>>(lay.G, parts, n, nnz, vis.ecap, ctl, d_out, g->rpb ? 1u : 0u);
  }
}

cq_status score_enqueue(cq_context* ctx, const cq_graph* g, const int32_t* labels, int32_t L, void* ws, size_t ws_bytes,
                        ScoreResultDev* d_out, const cq_per_community* per_comm, const cq_pair_table* pairs, bool timed) {
  if (!ctx) return CQ_E_INVALID_ARG;
  ctx->err[0] = 0;
  if (!g || !labels || !d_out) return fail(ctx, CQ_E_INVALID_ARG, "null graph, labels or output");
  if (L < 1) return fail(ctx, CQ_E_INVALID_ARG, "num_labels must be >= 1");
  if (g->nnz == 0) return fail(ctx, CQ_E_NO_EDGES, "graph has no edges");
  if (g->w && (int64_t)L > (int64_t)HASH_WORDS)
    return fail(ctx, CQ_E_INVALID_ARG, "weighted scoring supports up to %u label ids", HASH_WORDS);
  if (pairs && pairs->capacity > 0 && (!pairs->ci || !pairs->cj || !pairs->count))
    return fail(ctx, CQ_E_INVALID_ARG, "pair table with null arrays");
  const ScoreLayout lay = graph_score_layout(g, L);
  if (!ws || ws_bytes < lay.total)
    return fail(ctx, CQ_E_WORKSPACE, "workspace %zu bytes, need %zu", ws_bytes, lay.total);
  if (reinterpret_cast<uintptr_t>(ws) % WS_ALIGN) return fail(ctx, CQ_E_INVALID_ARG, "workspace not 16-byte aligned");
  if (lay.small)
    score_launch<uint16_t>(ctx, g, labels, L, ws, lay, d_out, per_comm, pairs, timed);
  else
    score_launch<uint32_t>(ctx, g, labels, L, ws, lay, d_out, per_comm, pairs, timed);
  return launch_status(ctx, "score launch");
}

template <class LT>
void compare_launch(cq_context* ctx, int32_t n, const int32_t* la, int32_t La, const int32_t* lb, int32_t Lb, void* ws,
                    const CmpLayout& lay, CmpResultDev* d_out, const cq_cell_table* cells, bool timed) {
  hipStream_t s = ctx->stream;
  Ctl* ctl = at<Ctl>(ws, lay.ctl);
  u32* A = at<u32>(ws, lay.A);
  u32* B = at<u32>(ws, lay.B);
  u32* start = at<u32>(ws, lay.start);
  u32* order = at<u32>(ws, lay.order);
  u32* COLMAX = at<u32>(ws, lay.COLMAX);
  u32* loc = at<u32>(ws, lay.loc);
  LT* CB = at<LT>(ws, lay.CB);
  const u32* PM = nullptr;
  {
    StageMark mk(ctx, ST_SETUP, timed);
    fill(reinterpret_cast<u32*>(ctl), sizeof(Ctl) / 4, 0, s);
    fill(at<u32>(ws, lay.wq), WQ_WORDS, 0, s);
    fill(COLMAX, (size_t)Lb, 0, s);
    if (!lay.privA) fill(at<u32>(ws, lay.SZ), 2 * (size_t)La, 0, s);
    if (!lay.privB) fill(B, (size_t)Lb, 0, s);
  }
  if (lay.privA) {
    u32* HN = at<u32>(ws, lay.HN);
    {
      StageMark mk(ctx, ST_NODE, timed);
      for (int64_t lb = 0; lb < La; lb += PRIV_MAX) {
        const int lr = (int)std::min<int64_t>(PRIV_MAX, La - lb);
        k_node_priv<false, uint32_t><<<lay.W, 1024, (size_t)lr * 4, s>>>(n, la, nullptr, nullptr, La, lay.chunk, HN, nullptr, loc,
                                                                         nullptr, ctl, (int)lb, lr);
      }
    }
    {
      StageMark mk(ctx, ST_COLSCAN, timed);
      k_colscan<false, true><<<colscan_grid(La), CS_LABELS * CS_GROUPS, 0, s>>>(lay.W, La, HN, HN, A, nullptr);
    }
    PM = HN;
  } else {
    unsigned long long* SZ = at<unsigned long long>(ws, lay.SZ);
    {
      StageMark mk(ctx, ST_NODE, timed);
      k_node_global<false, uint32_t><<<grid_for(n, 256, 8192), 256, 0, s>>>(n, la, nullptr, nullptr, La, SZ, loc, nullptr, ctl);
    }
    {
      StageMark mk(ctx, ST_COLSCAN, timed);
      k_unpack<<<grid_for(La, 256, 4096), 256, 0, s>>>(La, SZ, A, nullptr);
    }
  }
  {
    StageMark mk(ctx, ST_HIST_B, timed);
    if (lay.privB) {
      u32* HB = at<u32>(ws, lay.HB);
      for (int64_t b0 = 0; b0 < Lb; b0 += PRIV_MAX) {
        const int br = (int)std::min<int64_t>(PRIV_MAX, Lb - b0);
        k_hist_priv<<<lay.Wb, 1024, (size_t)br * 4, s>>>(n, lb, Lb, HB, ctl, (int)b0, br);
      }
      k_colscan<false, false><<<colscan_grid(Lb), CS_LABELS * CS_GROUPS, 0, s>>>(lay.Wb, Lb, HB, HB, B, nullptr);
    } else {
      k_hist_global<<<grid_for(n, 256, 8192), 256, 0, s>>>(n, lb, Lb, B, ctl);
    }
  }
  {
    StageMark mk(ctx, ST_ORDER, timed);
    k_scan_order<<<1, 1024, 0, s>>>(La, A, A, start, order, ctl);
  }
  {
    StageMark mk(ctx, ST_SCATTER, timed);
    if (lay.privA)
      k_cmp_scatter<true, LT><<<grid_for(n, 256, 8192), 256, 0, s>>>(n, la, lb, La, Lb, lay.chunk, PM, start, loc, CB);
    else
      k_cmp_scatter<false, LT><<<grid_for(n, 256, 8192), 256, 0, s>>>(n, la, lb, La, Lb, lay.chunk, PM, start, loc, CB);
  }
  CmpVis vis;
  vis.A = A;
  vis.B = B;
  vis.Nd = (double)n;
  vis.COLMAX = COLMAX;
  vis.RA11 = at<u64>(ws, lay.RA11);
  vis.RMAX = at<u32>(ws, lay.RMAX);
  vis.RF = at<double>(ws, lay.RF);
  vis.RXL = at<u64>(ws, lay.RXL);
  vis.eci = cells ? cells->ci : nullptr;
  vis.ecj = cells ? cells->cj : nullptr;
  vis.ecnt = cells ? cells->count : nullptr;
  vis.ecap = cells ? cells->capacity : 0;
  vis.ctl = ctl;
  vis.wq = at<u32>(ws, lay.wq);
  const u32 lds_words = Lb <= DIRECT_MAX ? std::max<u32>(((u32)Lb + 3u) & ~3u, 128u) : HASH_WORDS;
  const size_t lds = (size_t)lds_words * 4;
  {
    StageMark mk(ctx, ST_GROUPS, timed);
    // 16-bit labels: groups of fewer than GW_SPLIT entries are counted one per wave after
    // the workgroup-per-group pass has taken the larger ones
    constexpr bool waves = sizeof(LT) == 2;
    k_groups<CmpVis, LT><<<group_grid<CmpVis, LT>(ctx, lds), GBLOCK, lds, s>>>(CB, start, A, order, ctl, (u32)Lb, lds_words, vis,
                                                                               nullptr, vis.wq, waves);
    if constexpr (waves) {
      int nb = 0;
      if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_groups_wave<CmpVis>, 64 * GW_WAVES, 0) != hipSuccess || nb < 1) nb = 1;
      k_groups_wave<CmpVis><<<(unsigned)(ctx->num_cus * nb), 64 * GW_WAVES, 0, s>>>(CB, start, A, order, ctl, (u32)Lb, vis, vis.wq);
    }
  }
  CmpPart* parts = at<CmpPart>(ws, lay.parts);
  {
    StageMark mk(ctx, ST_FINAL, timed);
    k_cmp_final1<<<lay.Ga + lay.Gb, FBLOCK, 0, s>>>(La, Lb, lay.Ga, A, B, COLMAX, vis.RA11, vis.RMAX, vis.RF, vis.RXL,
                                                   (double)n, parts);
    k_cmp_final2<<<1, 64, 0, s>>>(lay.Ga + lay.Gb, parts, n, vis.ecap, ctl, d_out, vis.wq);
  }
}

// Per-label histogram of labels[0, n) (ranges of PRIV_MAX labels per launch) into totals N.
void label_totals(int n, const int32_t* labels, int L, int W, u32* H, u32* N, Ctl* ctl, hipStream_t s) {
  for (int64_t l0 = 0; l0 < L; l0 += PRIV_MAX) {
    const int lr = (int)std::min<int64_t>(PRIV_MAX, L - l0);
    k_hist_priv<<<W, 1024, (size_t)lr * 4, s>>>(n, labels, L, H, ctl, (int)l0, lr);
  }
  k_colscan<false, false><<<colscan_grid(L), CS_LABELS * CS_GROUPS, 0, s>>>(W, L, H, H, N, nullptr);
}

unsigned cells_grid(cq_context* ctx) {
  static int nb = 0;
  if (nb == 0 && (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_cmp_cells, CC_THREADS, 0) != hipSuccess || nb < 1))
    nb = 1;
  return (unsigned)(ctx->num_cus * nb);
}

// Both label spaces fit 16 bits: contingency cells counted per band of ground-truth labels.
void compare_launch_bands(cq_context* ctx, int32_t n, const int32_t* la, int32_t La, const int32_t* lb, int32_t Lb, void* ws,
                          const CmpLayout& lay, CmpResultDev* d_out, const cq_cell_table* cells, bool timed) {
  hipStream_t s = ctx->stream;
  Ctl* ctl = at<Ctl>(ws, lay.ctl);
  u32* A = at<u32>(ws, lay.A);
  u32* B = at<u32>(ws, lay.B);
  u32* COLMAX = at<u32>(ws, lay.COLMAX);
  u32* wq = at<u32>(ws, lay.wq);
  u32* sbk = at<u32>(ws, lay.sbk);
  u32* SBA = at<u32>(ws, lay.SBA);
  u32* SZB = at<u32>(ws, lay.SZB);
  u32* SBS = at<u32>(ws, lay.SBS);
  u32* CUR = at<u32>(ws, lay.CUR);
  u32* BORD = at<u32>(ws, lay.BORD);
  u32* E = at<u32>(ws, lay.E);
  u64* RA11 = at<u64>(ws, lay.RA11);
  u32* RMAX = at<u32>(ws, lay.RMAX);
  double* RF = at<double>(ws, lay.RF);
  u64* RXL = at<u64>(ws, lay.RXL);
  {
    StageMark mk(ctx, ST_SETUP, timed);
    const int words = (int)(sizeof(Ctl) / 4) + (int)WQ_WORDS + Lb;
    k_cmp_clear<<<grid_for(words, 256, 1024), 256, 0, s>>>(reinterpret_cast<u32*>(ctl), (int)(sizeof(Ctl) / 4), wq, COLMAX, Lb);
  }
  if ((int64_t)La + Lb <= 2 * PRIV_MAX) {
    StageMark mk(ctx, ST_NODE, timed);
    u32* HA = at<u32>(ws, lay.HA);
    u32* HB = at<u32>(ws, lay.HB);
    (void)hipFuncSetAttribute((const void*)k_hist2_priv, hipFuncAttributeMaxDynamicSharedMemorySize, (La + Lb) * 4);
    k_hist2_priv<<<lay.Wa, 1024, ((size_t)La + Lb) * 4, s>>>(n, la, La, lb, Lb, HA, HB, ctl);
    const int ga = (int)colscan_grid(La), gb = (int)colscan_grid(Lb);
    k_cmp_totals<<<ga + gb, CS_LABELS * CS_GROUPS, 0, s>>>(lay.Wa, La, Lb, ga, HA, HB, A, B);
  } else {
    {
      StageMark mk(ctx, ST_NODE, timed);
      label_totals(n, la, La, lay.Wa, at<u32>(ws, lay.HA), A, ctl, s);
    }
    {
      StageMark mk(ctx, ST_HIST_B, timed);
      label_totals(n, lb, Lb, lay.Wb, at<u32>(ws, lay.HB), B, ctl, s);
    }
  }
  {
    StageMark mk(ctx, ST_ORDER, timed);
    k_cmp_bands<<<1, 1024, 0, s>>>(La, A, lay.T, sbk, SBA, SBS, SZB, CUR, BORD, ctl);
  }
  {
    StageMark mk(ctx, ST_SCATTER, timed);
    (void)hipFuncSetAttribute((const void*)k_cmp_part, hipFuncAttributeMaxDynamicSharedMemorySize, lay.nbmax * 8);
    k_cmp_part<<<lay.Wc, CP_THREADS, (size_t)lay.nbmax * 8, s>>>(n, la, lb, La, Lb, sbk, lay.nbmax, lay.rounds, CUR, E);
  }
  const long long ecap = cells ? cells->capacity : 0;
  {
    StageMark mk(ctx, ST_GROUPS, timed);
    k_cmp_cells<<<cells_grid(ctx), CC_THREADS, 0, s>>>(E, SBS, SZB, SBA, BORD, ctl, A, B, (double)n, COLMAX, RA11, RMAX, RF,
                                                       RXL, cells ? cells->ci : nullptr, cells ? cells->cj : nullptr,
                                                       cells ? cells->count : nullptr, ecap, wq);
  }
  CmpPart* parts = at<CmpPart>(ws, lay.parts);
  {
    StageMark mk(ctx, ST_FINAL, timed);
    k_cmp_final1<<<lay.Ga + lay.Gb, FBLOCK, 0, s>>>(La, Lb, lay.Ga, A, B, COLMAX, RA11, RMAX, RF, RXL, (double)n, parts);
    k_cmp_final2<<<1, 64, 0, s>>>(lay.Ga + lay.Gb, parts, n, ecap, ctl, d_out, wq);
  }
}

cq_status compare_enqueue(cq_context* ctx, int32_t n, const int32_t* la, int32_t La, const int32_t* lb, int32_t Lb, void* ws,
                          size_t ws_bytes, CmpResultDev* d_out, const cq_cell_table* cells, bool timed) {
  if (!ctx) return CQ_E_INVALID_ARG;
  ctx->err[0] = 0;
  if (!la || !lb || !d_out) return fail(ctx, CQ_E_INVALID_ARG, "null labels or output");
  if (n < 2) return fail(ctx, CQ_E_INVALID_ARG, "n must be >= 2");
  if (La < 1 || Lb < 1) return fail(ctx, CQ_E_INVALID_ARG, "num_labels must be >= 1");
  if (cells && cells->capacity > 0 && (!cells->ci || !cells->cj || !cells->count))
    return fail(ctx, CQ_E_INVALID_ARG, "cell table with null arrays");
  const CmpLayout lay = cmp_layout(n, La, Lb);
  if (!ws || ws_bytes < lay.total)
    return fail(ctx, CQ_E_WORKSPACE, "workspace %zu bytes, need %zu", ws_bytes, lay.total);
  if (reinterpret_cast<uintptr_t>(ws) % WS_ALIGN) return fail(ctx, CQ_E_INVALID_ARG, "workspace not 16-byte aligned");
  if (lay.bands)
    compare_launch_bands(ctx, n, la, La, lb, Lb, ws, lay, d_out, cells, timed);
  else if (lay.small)
    compare_launch<uint16_t>(ctx, n, la, La, lb, Lb, ws, lay, d_out, cells, timed);
  else
    compare_launch<uint32_t>(ctx, n, la, La, lb, Lb, ws, lay, d_out, cells, timed);
  return launch_status(ctx, "compare launch");
}

template <class R>
cq_status fetch(cq_context* ctx, const void* d_res, R* h_out) {
  hipError_t e = hipMemcpyAsync(ctx->pinned, d_res, sizeof(R), hipMemcpyDeviceToHost, ctx->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
  if (e != hipSuccess) return fail(ctx, CQ_E_DEVICE, "result copy: %s", hipGetErrorString(e));
  std::memcpy(h_out, ctx->pinned, sizeof(R));
  if (ctx->timing) collect_stage_times(ctx);
  return CQ_OK;
}

void set_big_lds(const void* fn, size_t bytes) {
  (void)hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

// Exclusive scan of in[0, n) into out[0, n] (out[n] = total) using tmp tiles.
void scan_u32(const u32* in, u32* out, long long n, u32* tiles, hipStream_t s) {
  const int T = (int)((n + SCAN_TILE - 1) / SCAN_TILE);
  k_scan_tiles<<<std::max(T, 1), SCAN_THREADS, 0, s>>>(n, in, out, tiles);
  k_scan_tops<<<1, SCAN_THREADS, 0, s>>>(T, tiles, n, out);
  if (T > 0) k_scan_add<<<T, SCAN_THREADS, 0, s>>>(n, out, tiles);
}

constexpr int LP_SWEEPS = 10;
constexpr int LP_SALTED_SWEEPS = 20;
// Column blocks pay off while one block's labels (2 bytes per node) fit an XCD's L2, and
// once all labels do not (below that the plain edge pass has more workgroups in flight).
constexpr int64_t BLOCK_MAX_N = 16 << 20;
constexpr int64_t BLOCK_MIN_N = 1 << 20;

// Splits the renumbered graph (g->owned_rp / owned_col) into COL_BLOCKS column blocks.
cq_status build_column_blocks(cq_context* ctx, cq_graph* g) {
  const int n = g->n;
  const int64_t nnz = g->nnz;
  hipStream_t s = ctx->stream;
  const long long len = (long long)COL_BLOCKS * ((long long)n + 1);
  u32 *cnt = nullptr, *tiles = nullptr;
  hipError_t e = hipSuccess;
  auto alloc = [&](void** p, size_t bytes) {
    if (e == hipSuccess) e = hipMalloc(p, std::max<size_t>(bytes, 4));
  };
  alloc((void**)&g->rpb, 4 * ((size_t)len + 1));
  alloc((void**)&g->colb, 4 * (size_t)nnz);
  alloc((void**)&g->rowb, 4 * (size_t)nnz);
  if (g->owned_w) alloc((void**)&g->wb, 4 * (size_t)nnz);
  alloc((void**)&cnt, 4 * (size_t)len);
  alloc((void**)&tiles, 4 * ((size_t)((len + SCAN_TILE - 1) / SCAN_TILE) + 1));
  cq_status st = CQ_OK;
  if (e != hipSuccess) {
    st = fail(ctx, CQ_E_DEVICE, "allocating column blocks: %s", hipGetErrorString(e));
  } else {
    const int span = (int)(((int64_t)n + COL_BLOCKS - 1) / COL_BLOCKS);
    const unsigned gw = grid_for((int64_t)n * 64, 256, 65535);
    k_blk_count<<<gw, 256, 0, s>>>(n, g->owned_rp, g->owned_col, span, cnt);
    scan_u32(cnt, g->rpb, len, tiles, s);
    k_blk_place<<<gw, 256, 0, s>>>(n, g->owned_rp, g->owned_col, span, g->rpb, g->colb, g->rowb, g->owned_w, g->wb);
    e = hipGetLastError();
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    // far-entry ranges of every block: rows [0, s0) and [s1, n), s0..s1 being its span
    g->far_tiles = 0;
    const u32 ent = g->owned_w ? FT_ENT_W : FT_ENT;  // entries per far tile, as the gather kernel takes them
    for (int y = 0; y < COL_BLOCKS && e == hipSuccess; ++y) {
      const int64_t s0 = std::min<int64_t>(n, (int64_t)y * span), s1 = std::min<int64_t>(n, s0 + span);
      const int64_t at_row[4] = {0, s0, s1, n};
      for (int j = 0; j < 4 && e == hipSuccess; ++j)
        e = hipMemcpy(&g->far.b[y][j], g->rpb + (size_t)y * ((size_t)n + 1) + at_row[j], 4, hipMemcpyDeviceToHost);
      const u32 t = (g->far.b[y][1] - g->far.b[y][0] + ent - 1) / ent + (g->far.b[y][3] - g->far.b[y][2] + ent - 1) / ent;
      g->far_tiles = std::max(g->far_tiles, (unsigned)t);
    }
    if (e != hipSuccess) st = fail(ctx, CQ_E_DEVICE, "building column blocks: %s", hipGetErrorString(e));
  }
  if (cnt) (void)hipFree(cnt);
  if (tiles) (void)hipFree(tiles);
  if (st != CQ_OK) {
    if (g->rpb) (void)hipFree(g->rpb);
    if (g->colb) (void)hipFree(g->colb);
    if (g->rowb) (void)hipFree(g->rowb);
    if (g->wb) (void)hipFree(g->wb);
    g->rpb = nullptr;
    g->colb = nullptr;
    g->rowb = nullptr;
    g->wb = nullptr;
  }
  return st;
}

// Builds the label permutation plan of a renumbered graph from newid (caller id ->
// stored id) and the caller's row_ptr.
cq_status build_perm_plan(cq_context* ctx, cq_graph* g, const int32_t* newid, const int32_t* rp_in) {
  const int n = g->n;
  hipStream_t s = ctx->stream;
  const int nb = (int)(((int64_t)n + (1 << PERM_SHIFT) - 1) >> PERM_SHIFT);
  if (nb > PERM_MAX_BUCKETS) return CQ_OK;  // no plan: scoring gathers labels through perm instead
  u32 *bcnt = nullptr, *tiles = nullptr;
  hipError_t e = hipSuccess;
  auto alloc = [&](void** p, size_t bytes) {
    if (e == hipSuccess) e = hipMalloc(p, std::max<size_t>(bytes, 4));
  };
  alloc((void**)&g->deg_in, 4 * (size_t)n);
  alloc((void**)&g->pos1, 4 * (size_t)n);
  alloc((void**)&g->tgt, 2 * (size_t)n);
  alloc((void**)&g->pbstart, 4 * ((size_t)nb + 1));
  if (g->rpb) {
    alloc((void**)&g->lrank, 2 * (size_t)n);
    alloc((void**)&g->spos, 4 * (size_t)n);
  } else if (((int64_t)n + SB_MASK) >> SB_SHIFT <= SB_MAX) {
    alloc((void**)&g->sid, 4 * (size_t)n);
  }
  alloc((void**)&bcnt, 4 * ((size_t)nb + 1));
  u32* bstart = g->pbstart;
  alloc((void**)&tiles, 4 * ((size_t)((nb + SCAN_TILE - 1) / SCAN_TILE) + 1));
  cq_status st = CQ_OK;
  if (e != hipSuccess) {
    st = fail(ctx, CQ_E_DEVICE, "allocating the label permutation plan: %s", hipGetErrorString(e));
  } else {
    const unsigned gn = grid_for(n, 256, 8192);
    const unsigned gp = (unsigned)(((int64_t)n + PERM_NODES - 1) / PERM_NODES);
    k_degree<<<gn, 256, 0, s>>>(n, rp_in, g->deg_in);
    fill(bcnt, (size_t)nb + 1, 0, s);
    k_perm_count<<<gp, 256, 0, s>>>(n, newid, nb, bcnt);
    scan_u32(bcnt, bstart, nb, tiles, s);
    fill(bcnt, (size_t)nb + 1, 0, s);
    k_perm_plan<<<gp, 256, 8 * (size_t)nb, s>>>(n, newid, nb, bstart, bcnt, g->pos1, g->tgt, g->lrank, g->spos);
    if (g->sid) e = hipMemcpyAsync(g->sid, newid, 4 * (size_t)n, hipMemcpyDeviceToDevice, s);
    if (e == hipSuccess) e = hipGetLastError();
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) st = fail(ctx, CQ_E_DEVICE, "building the label permutation plan: %s", hipGetErrorString(e));
  }
  for (void* p : {(void*)bcnt, (void*)tiles})
    if (p) (void)hipFree(p);
  if (st != CQ_OK) {
    for (u32** p : {&g->deg_in, &g->pos1, &g->pbstart, &g->spos, &g->sid}) {
      if (*p) (void)hipFree(*p);
      *p = nullptr;
    }
    for (uint16_t** p : {&g->tgt, &g->lrank}) {
      if (*p) (void)hipFree(*p);
      *p = nullptr;
    }
  } else {
    g->perm_buckets = nb;
  }
  return st;
}

// Builds the renumbered copy of a graph (see CQ_GRAPH_REORDER in cq.h).
cq_status build_locality_order(cq_context* ctx, cq_graph* g, const int32_t* rp, const int32_t* col, bool blocks) {
  const int n = g->n;
  const int64_t nnz = g->nnz;
  hipStream_t s = ctx->stream;
  const size_t tiles_n = (size_t)((n + 1 + SCAN_TILE - 1) / SCAN_TILE) + 1;
  int32_t *lpA = nullptr, *lpB = nullptr, *newid = nullptr;
  u32 *cnt = nullptr, *start = nullptr, *tiles = nullptr;
  hipError_t e = hipSuccess;
  auto alloc = [&](void** p, size_t bytes) {
    if (e == hipSuccess) e = hipMalloc(p, std::max<size_t>(bytes, 4));
  };
  alloc((void**)&g->owned_rp, 4 * ((size_t)n + 1));
  alloc((void**)&g->owned_col, 4 * (size_t)std::max<int64_t>(nnz, 1));
  alloc((void**)&g->owned_perm, 4 * (size_t)n);
  if (g->w) alloc((void**)&g->owned_w, 4 * (size_t)std::max<int64_t>(nnz, 1));
  alloc((void**)&lpA, 4 * (size_t)n);
  alloc((void**)&lpB, 4 * (size_t)n);
  alloc((void**)&newid, 4 * (size_t)n);
  alloc((void**)&cnt, 4 * ((size_t)n + 1));
  alloc((void**)&start, 4 * ((size_t)n + 1));
  alloc((void**)&tiles, 4 * tiles_n);
  cq_status st = CQ_OK;
  if (e != hipSuccess) {
    st = fail(ctx, CQ_E_DEVICE, "allocating the renumbered graph: %s", hipGetErrorString(e));
  } else {
    const unsigned gw = grid_for((int64_t)n * 64, 256, 65535);  // one wave per row
    const unsigned gn = grid_for(n, 256, 8192);
    // Two label propagations: ties broken in one fixed order of labels (LP_SWEEPS sweeps),
    // and ties broken per node and sweep (LP_SALTED_SWEEPS).  The first settles fast on
    // sparse graphs; the second gives purer clusters where it converges.  The order uses
    // the one that ends with fewer clusters.
    u32 cs[2] = {0, 0};
    auto count_clusters = [&](const int32_t* lab) {
      fill(cnt, (size_t)n + 1, 0, s);
      k_count_labels<<<gn, 256, 0, s>>>(n, lab, cnt);
      fill(ctx->dscratch, 2, 0, s);
      k_cluster_stats<<<gn, 256, 0, s>>>(n, cnt, ctx->dscratch);
      if (e == hipSuccess) e = hipMemcpyAsync(cs, ctx->dscratch, 8, hipMemcpyDeviceToHost, s);
      if (e == hipSuccess) e = hipStreamSynchronize(s);
    };
    k_iota<<<gn, 256, 0, s>>>(n, lpA);
    for (int it = 0; it < LP_SWEEPS; ++it) {
      k_lp<<<gw, 256, 0, s>>>(n, rp, col, lpA, lpB, -1);
      std::swap(lpA, lpB);
    }
    count_clusters(lpA);
    const u32 plain_clusters = cs[0];
    int32_t* sa = lpB;  // newid is free until the nodes are placed
    int32_t* sb = newid;
    k_iota<<<gn, 256, 0, s>>>(n, sa);
    for (int it = 0; it < LP_SALTED_SWEEPS; ++it) {
      k_lp<<<gw, 256, 0, s>>>(n, rp, col, sa, sb, it);
      std::swap(sa, sb);
    }
    count_clusters(sa);
    if (cs[0] < plain_clusters) {
      // keep the salted labels in lpA; newid takes a free buffer
      if (sa == newid) std::swap(newid, lpA);
      else std::swap(lpB, lpA);
    } else {
      count_clusters(lpA);
    }
    g->clusters = cs[0];
    g->largest_cluster = cs[1];
    scan_u32(cnt, start, n, tiles, s);
    fill(cnt, (size_t)n + 1, 0, s);
    k_place<<<gn, 256, 0, s>>>(n, lpA, start, cnt, newid, g->owned_perm);
    k_new_degree<<<gn, 256, 0, s>>>(n, rp, g->owned_perm, cnt);
    scan_u32(cnt, reinterpret_cast<u32*>(g->owned_rp), n, tiles, s);
    k_relabel_rows<<<gw, 256, 0, s>>>(n, rp, col, g->owned_perm, newid, g->owned_rp, g->owned_col, g->w, g->owned_w);
    if (blocks) st = build_column_blocks(ctx, g);
    if (st == CQ_OK && (g->rpb || n >= BLOCK_MIN_N)) st = build_perm_plan(ctx, g, newid, rp);
    e = hipGetLastError();
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (st == CQ_OK && e != hipSuccess) st = fail(ctx, CQ_E_DEVICE, "renumbering the graph: %s", hipGetErrorString(e));
  }
  for (void* p : {(void*)lpA, (void*)lpB, (void*)newid, (void*)cnt, (void*)start, (void*)tiles})
    if (p) (void)hipFree(p);
  if (st == CQ_OK) {
    g->rp = g->owned_rp;
    g->col = g->owned_col;
    g->perm = g->owned_perm;
    if (g->owned_w) g->w = g->owned_w;
    g->reordered = CQ_GRAPH_REORDER | (g->rpb ? 0u : CQ_GRAPH_NO_BLOCKS);
    g->owned_bytes = (int64_t)(4 * ((size_t)n + 1) + 4 * (size_t)nnz + 4 * (size_t)n);
    if (g->rpb) g->owned_bytes += (int64_t)(4 * ((size_t)COL_BLOCKS * ((size_t)n + 1) + 1) + 8 * (size_t)nnz);
    if (g->pos1) g->owned_bytes += (int64_t)(10 * (size_t)n + 4 * ((size_t)g->perm_buckets + 1));
    if (g->lrank) g->owned_bytes += (int64_t)(6 * (size_t)n);
    if (g->sid) g->owned_bytes += (int64_t)(4 * (size_t)n);
    if (g->owned_w) g->owned_bytes += (int64_t)(4 * (size_t)nnz);
    if (g->wb) g->owned_bytes += (int64_t)(4 * (size_t)nnz);
  }
  return st;
}


// ---- batched scoring -------------------------------------------------------
constexpr int kGatherRows[3] = {128, 256, 512};
constexpr int64_t BATCH_MAX_L = PRIV_MAX;
constexpr int BATCH_MAX_TASKS = 1 << 18;  // the group pass's item list packs (task << 14) | group

void batch_launch(cq_batch_plan* p, hipStream_t s, int rsel, int occ) {
  const int T = (int)p->tasks.size();
  const TaskDev* td = static_cast<const TaskDev*>(p->td);
  const GroupDev* gd = static_cast<const GroupDev*>(p->gd);
  const int ng = (int)p->groups.size();
  k_b_setup<<<T, 64, 0, s>>>(T, td, p->wq);
  k_b_node<<<p->NXsum, 1024, 2 * (size_t)p->maxL * 4, s>>>(td, p->XWpre, p->XT, T);
  k_b_colscan<<<grid_for(p->Lsum, 256, 1u << 30), 256, 0, s>>>(td, p->Lpre, T);
  k_b_scan_order<<<T, 1024, 0, s>>>(td);
  k_b_kprefix<<<1, 1024, 0, s>>>(td, T, p->Kpre);
  k_b_items<<<(unsigned)(p->ctx->num_cus * 4), 256, 0, s>>>(td, p->Kpre, T, p->items);
  switch (rsel) {
    case 0: k_b_gather<128><<<p->RBsum[0], 128, 0, s>>>(gd, p->RBpre[0], p->XG[0], ng, td); break;
    case 1: k_b_gather<256><<<p->RBsum[1], 256, 0, s>>>(gd, p->RBpre[1], p->XG[1], ng, td); break;
    default: k_b_gather<512><<<p->RBsum[2], 512, 0, s>>>(gd, p->RBpre[2], p->XG[2], ng, td); break;
  }
  const u32 lds_words = std::max<u32>(((u32)p->maxL + 3u) & ~3u, 128u);
  // tasks of at most SMALL_L_MAX labels in 128-thread workgroups (twice the blocks per CU
  // of the tuned setting, within what fits), the others in 256-thread ones
  if (p->nsmall > 0) {
    int nb = 1;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_b_groups<GBLOCK_SMALL>, GBLOCK_SMALL, (size_t)lds_words * 4) !=
            hipSuccess || nb < 1)
      nb = 1;
    k_b_groups<GBLOCK_SMALL><<<(unsigned)(p->ctx->num_cus * std::min(2 * occ, nb)), GBLOCK_SMALL, (size_t)lds_words * 4, s>>>(
        td, p->Kpre, T, p->wq, lds_words, p->items, 1);
  }
  if (p->nsmall < T)
    k_b_groups<GBLOCK_DIRECT><<<(unsigned)(p->ctx->num_cus * occ), GBLOCK_DIRECT, (size_t)lds_words * 4, s>>>(
        td, p->Kpre, T, p->wq + WQ_WORDS, lds_words, p->items, 0);
  k_b_final1<<<p->Gsum, FBLOCK, 0, s>>>(td, p->Gpre, T);
  k_b_final2<<<grid_for(T, 64, 1u << 20), 64, 0, s>>>(td, T);
}


struct BatchTabLayout {
  size_t td, gd, W, L, G, K, tk, RB[3], XG[3], XW, XT, total;
};

BatchTabLayout batch_tab_layout(int T, int ng) {
  BatchTabLayout l{};
  Carve c;
  l.td = c.take(sizeof(TaskDev) * T);
  l.gd = c.take(sizeof(GroupDev) * ng);
  l.W = c.take(4 * (T + 1));
  l.L = c.take(4 * (T + 1));
  l.G = c.take(4 * (T + 1));
  l.K = c.take(4 * (T + 1));
  l.tk = c.take(2 * WQ_BYTES);  // work queues of the two group passes
  for (int r = 0; r < 3; ++r) {
    l.RB[r] = c.take(4 * 8 * ((size_t)ng + 1));
    l.XG[r] = c.take(4 * 16 * (size_t)std::max(ng, 1));  // groups, then first tiles
  }
  l.XW = c.take(4 * 8 * ((size_t)T + 1));
  l.XT = c.take(4 * 16 * (size_t)std::max(T, 1));  // tasks, then first chunks
  l.total = c.off;
  return l;
}

// Work items (graphs' tile lists, tasks' chunk lists) to XCDs: item k has cnt[k] blocks.
// An item with more than 1/16 of all blocks has them dealt to the eight XCDs in turn; the
// others go whole, largest first, each to the XCD with the fewest blocks so far, so that
// an item's random reads stay in one XCD's L2.  Writes, per XCD, the block prefix of its
// list (m + 1 values, padded with the total) to pre[x * (m + 1) ..] and its items, then
// their first blocks (bit 31: dealt, every 8th block), to lst[x * m ..] and
// lst[8 * m + x * m ..] (m = cnt.size(), at least 1 for the layout); returns the longest
// list's block count.
u32 xcd_lists(const std::vector<u32>& cnt, u32* pre_all, u32* lst) {
  const int m = (int)cnt.size();
  uint64_t all = 0;
  for (u32 c : cnt) all += c;
  struct Entry {
    int k;
    u32 first, count;
    bool dealt;
  };
  std::vector<std::vector<Entry>> lists(8);
  u32 load[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  std::vector<int> idx;
  for (int k = 0; k < m; ++k) {
    const u32 nt = cnt[k];
    if ((uint64_t)nt * 16 > all) {
      for (u32 xb = 0; xb < 8; ++xb) {
        const u32 c = nt > xb ? (nt - xb + 7) / 8 : 0u;
        if (c) {
          lists[xb].push_back({k, xb, c, true});
          load[xb] += c;
        }
      }
    } else {
      idx.push_back(k);
    }
  }
  std::stable_sort(idx.begin(), idx.end(), [&](int a, int b) { return cnt[a] > cnt[b]; });
  for (int k : idx) {
    const int xb = (int)(std::min_element(load, load + 8) - load);
    lists[xb].push_back({k, 0u, cnt[k], false});
    load[xb] += cnt[k];
  }
  const size_t gs = (size_t)std::max(m, 1);
  u32 xmax = 0;
  for (int xb = 0; xb < 8; ++xb) {
    u32* pre = pre_all + (size_t)xb * (m + 1);
    pre[0] = 0;
    for (int j = 0; j < m; ++j) {
      const bool in = j < (int)lists[xb].size();
      const Entry e = in ? lists[xb][j] : Entry{0, 0u, 0u, false};
      lst[(size_t)xb * gs + j] = (u32)e.k;
      lst[8 * gs + (size_t)xb * gs + j] = e.first | (e.dealt ? 0x80000000u : 0u);
      pre[j + 1] = pre[j] + e.count;
    }
    xmax = std::max(xmax, pre[m]);
  }
  return xmax;
}

// Writes the device tables of plan p (task descriptors, group descriptors, block
// prefix tables) into the host blob hb, laid out as they will sit at d_tab, and points
// the plan at d_tab.  The caller copies hb to d_tab before the plan runs.
void batch_fill_tables(cq_batch_plan* p, void* d_ws, cq_score_result* d_results, char* hb, void* d_tab) {
  const int T = (int)p->tasks.size();
  const int ng = (int)p->groups.size();
  const BatchTabLayout tl = batch_tab_layout(T, ng);
  TaskDev* td = reinterpret_cast<TaskDev*>(hb + tl.td);
  GroupDev* gd = reinterpret_cast<GroupDev*>(hb + tl.gd);
  u32* Wpre = reinterpret_cast<u32*>(hb + tl.W);
  u32* Lpre = reinterpret_cast<u32*>(hb + tl.L);
  u32* Gpre = reinterpret_cast<u32*>(hb + tl.G);
  u32* Kpre = reinterpret_cast<u32*>(hb + tl.K);
  Wpre[0] = Lpre[0] = Gpre[0] = 0;
  for (int t = 0; t <= T; ++t) Kpre[t] = 0;
  std::memset(hb + tl.tk, 0, 2 * WQ_BYTES);
  for (int t = 0; t < T; ++t) {
    const cq_batch_task& bt = p->tasks[t];
    const cq_graph* g = bt.graph;
    const ScoreLayout lay = batch_task_layout(g->n, g->nnz, bt.num_labels);
    char* base = static_cast<char*>(d_ws) + p->ws_off[t];
    TaskDev d;
    std::memset(&d, 0, sizeof(d));
    d.labels = bt.d_labels;
    d.perm = g->perm;
    d.rp = g->rp;
    d.col = g->col;
    d.nnz = g->nnz;
    d.n = g->n;
    d.L = bt.num_labels;
    d.chunk = lay.chunk;
    d.W = lay.W;
    d.G = lay.G;
    d.ctl = reinterpret_cast<Ctl*>(base + lay.ctl);
    d.N = reinterpret_cast<u32*>(base + lay.N);
    d.D = reinterpret_cast<u32*>(base + lay.D);
    d.start = reinterpret_cast<u32*>(base + lay.start);
    d.order = reinterpret_cast<u32*>(base + lay.order);
    d.I = reinterpret_cast<u32*>(base + lay.I);
    d.NP = reinterpret_cast<u32*>(base + lay.NP);
    d.PEN = reinterpret_cast<u64*>(base + lay.PEN);
    d.loc = reinterpret_cast<u32*>(base + lay.loc);
    d.HN = reinterpret_cast<u32*>(base + lay.HN);
    d.HD = reinterpret_cast<u32*>(base + lay.HD);
    d.labx = reinterpret_cast<uint16_t*>(base + lay.labx);  // replaced by the task's lane of its group below
    d.lst = 1;
    d.CB = reinterpret_cast<uint16_t*>(base + lay.CB);
    d.parts = reinterpret_cast<ScorePart*>(base + lay.parts);
    d.out = reinterpret_cast<ScoreResultDev*>(d_results + t);
    std::memcpy(&td[t], &d, sizeof(d));
    Wpre[t + 1] = Wpre[t] + (u32)lay.W;
    Lpre[t + 1] = Lpre[t] + (u32)bt.num_labels;
    Gpre[t + 1] = Gpre[t] + (u32)lay.G;
  }
  std::vector<int64_t> gn(ng);
  for (int k = 0; k < ng; ++k) {
    const cq_graph* g = p->tasks[p->groups[k][0]].graph;
    GroupDev gdv;
    std::memset(&gdv, 0, sizeof(gdv));
    gdv.rp = g->rp;
    gdv.col = g->col;
    gdv.n = g->n;
    gdv.np = p->group_np[k];
    for (int i = 0; i < BATCH_FUSE; ++i) gdv.task[i] = p->groups[k][i];
    gdv.il = reinterpret_cast<unsigned long long*>(static_cast<char*>(d_ws) + p->il_off[k]);
    std::memcpy(&gd[k], &gdv, sizeof(gdv));
    // the node pass writes task i's labels to lane i of the group's interleaved words
    for (int i = 0; i < gdv.np; ++i) {
      td[gdv.task[i]].labx = reinterpret_cast<uint16_t*>(gdv.il) + i;
      td[gdv.task[i]].lst = BATCH_FUSE;
    }
    gn[k] = g->n;
  }
  // groups to XCDs, per gather tile size: a group with more than 1/16 of all tiles has
  // its tiles dealt to the eight XCDs in turn; the others go whole, largest first, each to
  // the XCD with the fewest tiles so far (the edge pass then reads a graph's labels from
  // one XCD's L2)
  u32 xmax[3] = {0, 0, 0};
  for (int r = 0; r < 3; ++r) {
    const int R = kGatherRows[r];
    std::vector<u32> tiles(ng);
    for (int k = 0; k < ng; ++k) tiles[k] = (u32)((gn[k] + R - 1) / R);
    xmax[r] = xcd_lists(tiles, reinterpret_cast<u32*>(hb + tl.RB[r]), reinterpret_cast<u32*>(hb + tl.XG[r]));
  }
  // the node pass's chunks, by task, the same way
  std::vector<u32> chunks(T);
  for (int t = 0; t < T; ++t) chunks[t] = Wpre[t + 1] - Wpre[t];
  const u32 xmaxw = xcd_lists(chunks, reinterpret_cast<u32*>(hb + tl.XW), reinterpret_cast<u32*>(hb + tl.XT));
  char* b = static_cast<char*>(d_tab);
  p->td = b + tl.td;
  p->gd = b + tl.gd;
  p->Wpre = reinterpret_cast<u32*>(b + tl.W);
  p->Lpre = reinterpret_cast<u32*>(b + tl.L);
  p->Gpre = reinterpret_cast<u32*>(b + tl.G);
  p->Kpre = reinterpret_cast<u32*>(b + tl.K);
  p->wq = reinterpret_cast<u32*>(b + tl.tk);
  for (int r = 0; r < 3; ++r) {
    p->RBpre[r] = reinterpret_cast<u32*>(b + tl.RB[r]);
    p->XG[r] = reinterpret_cast<u32*>(b + tl.XG[r]);
    p->RBsum[r] = 8u * xmax[r];  // the gather grid: eight XCD lanes of the longest list
  }
  p->XWpre = reinterpret_cast<u32*>(b + tl.XW);
  p->XT = reinterpret_cast<u32*>(b + tl.XT);
  p->NXsum = 8u * xmaxw;
  p->Wsum = Wpre[T];
  p->Lsum = Lpre[T];
  p->Gsum = Gpre[T];
  p->ws = d_ws;
  p->items = reinterpret_cast<uint4*>(static_cast<char*>(d_ws) + p->items_off);
  p->d_results = d_results;
}

// Lays out a plan's per-task workspace and its groups (tasks already in p->tasks).
void batch_layout(cq_batch_plan* p) {
  p->ws_off.clear();
  p->groups.clear();
  p->group_np.clear();
  p->maxL = 1;
  p->nsmall = 0;
  Carve c;
  size_t labels_total = 0;
  for (const auto& t : p->tasks) {
    const ScoreLayout lay = batch_task_layout(t.graph->n, t.graph->nnz, t.num_labels);
    p->ws_off.push_back(c.take(lay.total));
    p->maxL = std::max(p->maxL, (int)t.num_labels);
    if ((u32)t.num_labels <= SMALL_L_MAX) ++p->nsmall;
    labels_total += (size_t)t.num_labels;
  }
  p->items_off = c.take(16 * labels_total);  // at most one item per label id of every task
  std::map<const cq_graph*, int> open;
  for (int i = 0; i < (int)p->tasks.size(); ++i) {
    auto it = open.find(p->tasks[i].graph);
    if (it == open.end() || p->group_np[it->second] == BATCH_FUSE) {
      p->groups.push_back({-1, -1, -1, -1});
      p->group_np.push_back(0);
      open[p->tasks[i].graph] = (int)p->groups.size() - 1;
      it = open.find(p->tasks[i].graph);
    }
    p->groups[it->second][p->group_np[it->second]++] = i;
  }
  p->il_off.clear();
  for (const auto& g : p->groups) p->il_off.push_back(c.take(8 * (size_t)p->tasks[g[0]].graph->n));
  p->ws_total = c.off;
}

int batch_max_occ(cq_batch_plan* p) {
  const u32 lds_words = std::max<u32>(((u32)p->maxL + 3u) & ~3u, 128u);
  int nb = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_b_groups<GBLOCK_DIRECT>, GBLOCK_DIRECT, (size_t)lds_words * 4) !=
          hipSuccess ||
      nb < 1)
    nb = 1;
  return nb;
}

std::string batch_key(const cq_batch_plan* p) {
  long long sn = 0, snnz = 0;
  for (const auto& t : p->tasks) {
    sn += t.graph->n;
    snnz += t.graph->nnz;
  }
  char buf[160];
  snprintf(buf, sizeof(buf), "gfx950:cus%d:T%zu:G%zu:n%lld:nnz%lld:L%d", p->ctx->num_cus, p->tasks.size(), p->groups.size(),
           sn, snnz, p->maxL);
  return buf;
}

std::mutex g_tune_mu;
std::map<std::string, std::array<double, 3>> g_tune;  // key -> (rsel, occ, ms)

// Tuning cache: kept for the process; when CQ_TUNE_CACHE names a file, it is also read
// from and appended to as JSON lines {"key": ..., "gather_rows": ..., "occ": ..., "ms": ...}.
bool tune_lookup(const std::string& key, int* rsel, int* occ, double* ms) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  const char* path = std::getenv("CQ_TUNE_CACHE");
  if (path && *path) {
    if (FILE* f = fopen(path, "r")) {
      char line[512];
      while (fgets(line, sizeof(line), f)) {
        char k[256];
        int rows = 0, o = 0;
        double t = 0;
        if (sscanf(line, "{\"key\": \"%255[^\"]\", \"gather_rows\": %d, \"occ\": %d, \"ms\": %lf}", k, &rows, &o, &t) == 4) {
          int r = rows == 128 ? 0 : rows == 256 ? 1 : 2;
          g_tune[k] = {(double)r, (double)o, t};
        }
      }
      fclose(f);
    }
  }
  auto it = g_tune.find(key);
  if (it == g_tune.end()) return false;
  *rsel = (int)it->second[0];
  *occ = (int)it->second[1];
  *ms = it->second[2];
  return true;
}

void tune_store(const std::string& key, int rsel, int occ, double ms) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  g_tune[key] = {(double)rsel, (double)occ, ms};
  const char* path = std::getenv("CQ_TUNE_CACHE");
  if (path && *path) {
    if (FILE* f = fopen(path, "a")) {
      fprintf(f, "{\"key\": \"%s\", \"gather_rows\": %d, \"occ\": %d, \"ms\": %.6f}\n", key.c_str(), kGatherRows[rsel], occ, ms);
      fclose(f);
    }
  }
}


// ---- serving -------------------------------------------------------------------
// The scheduler (request table, arena admission in arrival order, grouping of small
// scoring requests, waiting, shutdown) is host code in srv_core.hpp.  This executor runs
// what it admits on the device: one HIP stream per slot, the labels copied up from the
// caller's host memory, the scoring, comparison or batched kernels enqueued, the results
// copied back into pinned memory, and an event that tells when the slot is done.

struct SrvSlot {
  cq_context* ctx = nullptr;  // context bound to this slot's stream
  hipStream_t stream = nullptr;
  hipEvent_t ev = nullptr;
  char* pinned = nullptr;     // results, then the batch table blob
  size_t res_bytes = 0;
  void* d_tab = nullptr;
  cq_batch_plan plan;         // reused host plan for grouped launches (no HIP graph)
};

using cqsrv::aup;

cq_status status_of_flags(u32 f) {
  if (f & F_LABEL) return CQ_E_LABEL_RANGE;
  if (f & (F_STACK | F_SEGMENT)) return CQ_E_DEVICE;
  if (f & F_EXPORT) return CQ_E_CAPACITY;
  return CQ_OK;
}

class HipExecutor final : public cqsrv::Executor {
 public:
  int device = 0;
  char* arena = nullptr;  // device memory of memory_budget bytes
  std::vector<SrvSlot*> slots;

  void worker_init() override { (void)hipSetDevice(device); }

  // Labels at the start of the region, then the workspace, then the result.  A group of
  // small scoring requests runs as one batched launch: every request's labels, the
  // batch workspace, the results.
  void dispatch(int slot, const std::vector<cqsrv::Req*>& reqs, bool grouped, size_t off, size_t) override {
    SrvSlot* sl = slots[slot];
    hipStream_t st = sl->stream;
    char* region = arena + off;
    if (!grouped) {
      cqsrv::Req* r = reqs[0];
      if (r->kind == 0) {
        int32_t* d_lab = reinterpret_cast<int32_t*>(region);
        char* d_ws = region + aup(4 * (size_t)r->n);
        ScoreResultDev* d_res = reinterpret_cast<ScoreResultDev*>(d_ws + aup(r->ws_bytes));
        (void)hipMemcpyAsync(d_lab, r->ha, 4 * (size_t)r->n, hipMemcpyHostToDevice, st);
        r->status = score_enqueue(sl->ctx, static_cast<const cq_graph*>(r->graph), d_lab, r->L, d_ws, r->ws_bytes, d_res,
                                  nullptr, nullptr, false);
        (void)hipMemcpyAsync(sl->pinned, d_res, sizeof(cq_score_result), hipMemcpyDeviceToHost, st);
      } else {
        int32_t* d_a = reinterpret_cast<int32_t*>(region);
        int32_t* d_b = reinterpret_cast<int32_t*>(region + aup(4 * (size_t)r->n));
        char* d_ws = region + 2 * aup(4 * (size_t)r->n);
        CmpResultDev* d_res = reinterpret_cast<CmpResultDev*>(d_ws + aup(r->ws_bytes));
        (void)hipMemcpyAsync(d_a, r->ha, 4 * (size_t)r->n, hipMemcpyHostToDevice, st);
        (void)hipMemcpyAsync(d_b, r->hb, 4 * (size_t)r->n, hipMemcpyHostToDevice, st);
        r->status = compare_enqueue(sl->ctx, r->n, d_a, r->La, d_b, r->Lb, d_ws, r->ws_bytes, d_res, nullptr, false);
        (void)hipMemcpyAsync(sl->pinned, d_res, sizeof(cq_compare_result), hipMemcpyDeviceToHost, st);
      }
    } else {
      cq_batch_plan* p = &sl->plan;
      p->tasks.clear();
      size_t o = 0;
      for (cqsrv::Req* r : reqs) {
        int32_t* d_lab = reinterpret_cast<int32_t*>(region + o);
        (void)hipMemcpyAsync(d_lab, r->ha, 4 * (size_t)r->n, hipMemcpyHostToDevice, st);
        p->tasks.push_back({static_cast<const cq_graph*>(r->graph), d_lab, r->L});
        o += aup(4 * (size_t)r->n);
      }
      batch_layout(p);
      char* d_ws = region + o;
      cq_score_result* d_res = reinterpret_cast<cq_score_result*>(d_ws + aup(p->ws_total));
      const BatchTabLayout tl = batch_tab_layout((int)p->tasks.size(), (int)p->groups.size());
      char* blob = sl->pinned + sl->res_bytes;
      batch_fill_tables(p, d_ws, d_res, blob, sl->d_tab);
      (void)hipMemcpyAsync(sl->d_tab, blob, tl.total, hipMemcpyHostToDevice, st);
      batch_launch(p, st, 1, batch_max_occ(p));
      (void)hipMemcpyAsync(sl->pinned, d_res, sizeof(cq_score_result) * p->tasks.size(), hipMemcpyDeviceToHost, st);
    }
    (void)hipEventRecord(sl->ev, st);
  }

  bool finished(int slot) override { return hipEventQuery(slots[slot]->ev) == hipSuccess; }

  void collect(int slot, const std::vector<cqsrv::Req*>& reqs, bool) override {
    const SrvSlot* sl = slots[slot];
    for (size_t i = 0; i < reqs.size(); ++i) {
      cqsrv::Req* r = reqs[i];
      if (r->status != CQ_OK) continue;  // never started
      if (r->kind == 0) {
        std::memcpy(&r->sres, sl->pinned + i * sizeof(cq_score_result), sizeof(cq_score_result));
        r->status = status_of_flags(r->sres.device_flags);
      } else {
        std::memcpy(&r->cres, sl->pinned, sizeof(cq_compare_result));
        r->status = status_of_flags(r->cres.device_flags);
      }
    }
  }
};

}  // namespace

struct cq_server {
  cq_context* ctx = nullptr;
  cq_server_config cfg{};
  HipExecutor exec;
  cqsrv::Scheduler* sched = nullptr;
};

static cq_status srv_submit(cq_server* srv, cqsrv::Req* r, uint64_t* ticket) {
  const char* why = nullptr;
  const size_t foot = cqsrv::req_footprint(*r);
  const cq_status st = srv->sched->submit(r, ticket, &why);
  if (st == CQ_E_BUSY)
    return fail(srv->ctx, st, "request needs %zu bytes, the server arena has %lld", foot, (long long)srv->cfg.memory_budget);
  if (st != CQ_OK) return fail(srv->ctx, st, "%s", why ? why : "request not queued");
  return CQ_OK;
}

extern "C" {

const char* cq_status_string(cq_status s) {
  switch (s) {
    case CQ_OK: return "CQ_OK";
    case CQ_E_INVALID_ARG: return "CQ_E_INVALID_ARG";
    case CQ_E_LABEL_RANGE: return "CQ_E_LABEL_RANGE";
    case CQ_E_GRAPH_FORMAT: return "CQ_E_GRAPH_FORMAT";
    case CQ_E_OVERFLOW: return "CQ_E_OVERFLOW";
    case CQ_E_WORKSPACE: return "CQ_E_WORKSPACE";
    case CQ_E_NO_EDGES: return "CQ_E_NO_EDGES";
    case CQ_E_DEVICE: return "CQ_E_DEVICE";
    case CQ_E_BUSY: return "CQ_E_BUSY";
    case CQ_E_CANCELLED: return "CQ_E_CANCELLED";
    case CQ_E_CAPACITY: return "CQ_E_CAPACITY";
    default: return "CQ_E_UNKNOWN";
  }
}

cq_status cq_context_create(int device, void* hip_stream, cq_context** out) {
  if (!out) return CQ_E_INVALID_ARG;
  *out = nullptr;
  int count = 0;
  if (hipGetDeviceCount(&count) != hipSuccess || device < 0 || device >= count) return CQ_E_DEVICE;
  if (hipSetDevice(device) != hipSuccess) return CQ_E_DEVICE;
  cq_context* ctx = new (std::nothrow) cq_context();
  if (!ctx) return CQ_E_DEVICE;
  ctx->device = device;
  ctx->stream = static_cast<hipStream_t>(hip_stream);
  ctx->scratch = scratch_address(device);  // null if the symbol lookup fails (noalloc calls then refuse)
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, device) == hipSuccess) ctx->num_cus = prop.multiProcessorCount;
  if (hipHostMalloc(&ctx->pinned, 4096, hipHostMallocDefault) != hipSuccess ||
      hipMalloc(&ctx->dscratch, 256) != hipSuccess) {
    if (ctx->pinned) (void)hipHostFree(ctx->pinned);
    delete ctx;
    return CQ_E_DEVICE;
  }
  for (int i = 0; i < 2 * CQ_MAX_STAGES; ++i) {
    if (hipEventCreate(&ctx->ev[i]) != hipSuccess) {
      cq_context_destroy(ctx);
      return CQ_E_DEVICE;
    }
  }
  const size_t gl = std::max<size_t>(DIRECT_MAX, HASH_WORDS) * 4;
  set_big_lds(reinterpret_cast<const void*>(k_node_priv<true, uint16_t>), 2 * PRIV_MAX * 4);
  set_big_lds(reinterpret_cast<const void*>(k_node_perm<uint16_t>), 2 * PRIV_MAX * 4);
  set_big_lds(reinterpret_cast<const void*>(k_node_perm<uint32_t>), 2 * PRIV_MAX * 4);
  set_big_lds(reinterpret_cast<const void*>(k_perm_apply<uint16_t>), ((size_t)1 << PERM_SHIFT) * 2);
  set_big_lds(reinterpret_cast<const void*>(k_perm_apply<uint32_t>), ((size_t)1 << PERM_SHIFT) * 4);
  set_big_lds(reinterpret_cast<const void*>(k_node_priv<true, uint32_t>), 2 * PRIV_MAX * 4);
  set_big_lds(reinterpret_cast<const void*>(k_node_priv<true, uint16_t, true>), 2 * PRIV_MAX * 4);
  set_big_lds(reinterpret_cast<const void*>(k_node_priv<true, uint32_t, true>), 2 * PRIV_MAX * 4);
  set_big_lds(reinterpret_cast<const void*>(k_node_priv<false, uint32_t>), PRIV_MAX * 4);
  set_big_lds(reinterpret_cast<const void*>(k_hist_priv), PRIV_MAX * 4);
  set_big_lds(reinterpret_cast<const void*>(k_perm_plan), 8 * (size_t)PERM_MAX_BUCKETS);
  set_big_lds(reinterpret_cast<const void*>(k_perm_apply_count), ((size_t)1 << PERM_SHIFT) * 2 + 8 * (size_t)APPLY_COUNT_MAX_L);
  set_big_lds(reinterpret_cast<const void*>(k_groups<ScoreVis, uint16_t, GBLOCK_WIDE>), gl);
  set_big_lds(reinterpret_cast<const void*>(k_groups_w<uint16_t>), gl);
  set_big_lds(reinterpret_cast<const void*>(k_groups_w<uint32_t>), gl);
  set_big_lds(reinterpret_cast<const void*>(k_groups<ScoreVis, uint32_t, GBLOCK_WIDE>), gl);
  set_big_lds(reinterpret_cast<const void*>(k_groups<CmpVis, uint16_t>), gl);
  set_big_lds(reinterpret_cast<const void*>(k_groups<CmpVis, uint32_t>), gl);
  set_big_lds(reinterpret_cast<const void*>(k_b_node), 2 * PRIV_MAX * 4);
  set_big_lds(reinterpret_cast<const void*>(k_b_groups<GBLOCK_DIRECT>), gl);
  set_big_lds(reinterpret_cast<const void*>(k_b_groups<GBLOCK_SMALL>), gl);
  *out = ctx;
  return CQ_OK;
}

cq_status cq_context_set_stream(cq_context* ctx, void* hip_stream) {
  if (!ctx) return CQ_E_INVALID_ARG;
  ctx->stream = static_cast<hipStream_t>(hip_stream);
  return CQ_OK;
}

void cq_context_destroy(cq_context* ctx) {
  if (!ctx) return;
  if (ctx->pinned) (void)hipHostFree(ctx->pinned);
  if (ctx->dscratch) (void)hipFree(ctx->dscratch);
  for (int i = 0; i < 2 * CQ_MAX_STAGES; ++i)
    if (ctx->ev[i]) (void)hipEventDestroy(ctx->ev[i]);
  delete ctx;
}

cq_status cq_context_time_stages(cq_context* ctx, uint32_t stage_mask) {
  if (!ctx) return CQ_E_INVALID_ARG;
  ctx->timing = stage_mask & ((1u << ST_COUNT) - 1u);
  for (int i = 0; i < CQ_MAX_STAGES; ++i) {
    ctx->total_ms[i] = 0.0;
    ctx->counts[i] = 0;
    ctx->recorded[i] = false;
  }
  return CQ_OK;
}

cq_status cq_context_set_row_staging(cq_context* ctx, double change_fraction) {
  if (!ctx) return CQ_E_INVALID_ARG;
  if (!(change_fraction == change_fraction)) return fail(ctx, CQ_E_INVALID_ARG, "change_fraction is NaN");
  ctx->row_staging_from = change_fraction;
  return CQ_OK;
}

cq_status cq_context_enable_timing(cq_context* ctx, int enable) {
  return cq_context_time_stages(ctx, enable ? ~0u : 0u);
}

cq_status cq_context_stage_times(const cq_context* ctx, double* total_ms, int64_t* counts, int32_t max_stages) {
  if (!ctx || !total_ms || !counts || max_stages < 0) return CQ_E_INVALID_ARG;
  for (int i = 0; i < max_stages && i < CQ_MAX_STAGES; ++i) {
    total_ms[i] = ctx->total_ms[i];
    counts[i] = ctx->counts[i];
  }
  return CQ_OK;
}

const char* cq_stage_name(int32_t s) { return (s >= 0 && s < ST_COUNT) ? kStageNames[s] : ""; }

const char* cq_context_last_error(const cq_context* ctx) { return ctx ? ctx->err : "null context"; }

namespace {
// Shared by the unweighted and weighted loads; d_weights may be null.
cq_status graph_load(cq_context* ctx, int32_t n, int64_t nnz, const int32_t* d_row_ptr, const int32_t* d_col_idx,
                     const float* d_weights, uint32_t flags, cq_graph** out) {
  if (!ctx) return CQ_E_INVALID_ARG;
  ctx->err[0] = 0;
  if (!out || !d_row_ptr || (nnz > 0 && !d_col_idx)) return fail(ctx, CQ_E_INVALID_ARG, "null pointer");
  *out = nullptr;
  if (n < 1) return fail(ctx, CQ_E_INVALID_ARG, "n must be >= 1");
  if (flags & ~(CQ_VALIDATE_GRAPH | CQ_GRAPH_REORDER | CQ_GRAPH_NO_BLOCKS | CQ_GRAPH_BLOCKS))
    return fail(ctx, CQ_E_INVALID_ARG, "unknown flag bits");
  if ((flags & (CQ_GRAPH_NO_BLOCKS | CQ_GRAPH_BLOCKS)) && !(flags & CQ_GRAPH_REORDER))
    return fail(ctx, CQ_E_INVALID_ARG, "CQ_GRAPH_NO_BLOCKS and CQ_GRAPH_BLOCKS need CQ_GRAPH_REORDER");
  if ((flags & CQ_GRAPH_NO_BLOCKS) && (flags & CQ_GRAPH_BLOCKS))
    return fail(ctx, CQ_E_INVALID_ARG, "CQ_GRAPH_NO_BLOCKS and CQ_GRAPH_BLOCKS exclude each other");
  if (nnz < 0 || nnz >= (int64_t)1 << 31) return fail(ctx, CQ_E_OVERFLOW, "nnz must be in [0, 2^31)");
  if (nnz % 2) return fail(ctx, CQ_E_GRAPH_FORMAT, "an undirected CSR stores an even number of entries");
  hipStream_t s = ctx->stream;
  int32_t ends[2] = {0, 0};
  hipError_t e = hipMemcpyAsync(&ends[0], d_row_ptr, 4, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipMemcpyAsync(&ends[1], d_row_ptr + n, 4, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return fail(ctx, CQ_E_DEVICE, "reading row_ptr: %s", hipGetErrorString(e));
  if (ends[0] != 0 || (int64_t)ends[1] != nnz) return fail(ctx, CQ_E_GRAPH_FORMAT, "row_ptr[0] != 0 or row_ptr[n] != nnz");
  fill(ctx->dscratch, 2 + DEG_BINS, 0, s);
  k_check_csr<<<grid_for(std::max<int64_t>(n, nnz), 256, 4096), 256, 0, s>>>(n, nnz, d_row_ptr, d_col_idx, ctx->dscratch,
                                                                            ctx->dscratch + 1, ctx->dscratch + 2);
  u32 res[2 + DEG_BINS] = {};
  e = hipMemcpyAsync(res, ctx->dscratch, sizeof(res), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return fail(ctx, CQ_E_DEVICE, "graph check: %s", hipGetErrorString(e));
  if (res[0]) return fail(ctx, CQ_E_GRAPH_FORMAT, "row_ptr not monotone or col_idx out of range");
  uint32_t validated = 0;
  // weighted graphs are always checked in full: the two entries of an edge must carry
  // the same weight (W and every weighted sum count each edge once from its two halves),
  // and that check needs sorted, symmetric rows
  if ((flags & CQ_VALIDATE_GRAPH) || d_weights) {
    fill(ctx->dscratch, 1, 0, s);
    k_check_symmetric<<<grid_for(n, 4, 8192), 256, 0, s>>>(n, d_row_ptr, d_col_idx, d_weights, ctx->dscratch);
    u32 f = 0;
    e = hipMemcpyAsync(&f, ctx->dscratch, 4, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return fail(ctx, CQ_E_DEVICE, "symmetry check: %s", hipGetErrorString(e));
    if (f) return fail(ctx, CQ_E_GRAPH_FORMAT,
                       d_weights ? "graph is not a simple symmetric CSR with sorted rows and equal weights on both "
                                   "entries of every edge"
                                 : "graph is not a simple symmetric CSR with sorted rows");
    validated = CQ_VALIDATE_GRAPH;
  }
  double total_w = 0.0;
  if (d_weights && nnz > 0) {
    // every weight in range, and W = (sum of all entries) / 2 summed exactly
    const unsigned gb = grid_for(nnz, 256, 1024);
    u64* parts = nullptr;
    e = hipMalloc((void**)&parts, 16 * (size_t)gb);
    if (e != hipSuccess) return fail(ctx, CQ_E_DEVICE, "allocating the weight sums: %s", hipGetErrorString(e));
    std::vector<u64> hp(2 * (size_t)gb);
    fill(ctx->dscratch, 1, 0, s);
    k_check_weights<<<gb, 256, 0, s>>>(nnz, d_weights, ctx->dscratch, parts);
    u32 f = 0;
    e = hipGetLastError();
    if (e == hipSuccess) e = hipMemcpyAsync(&f, ctx->dscratch, 4, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipMemcpyAsync(hp.data(), parts, 16 * (size_t)gb, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    (void)hipFree(parts);
    if (e != hipSuccess) return fail(ctx, CQ_E_DEVICE, "weight check: %s", hipGetErrorString(e));
    if (f) return fail(ctx, CQ_E_GRAPH_FORMAT, "edge weights must be finite and in [2^-32, 2^32]");
    u128 t = 0;
    for (unsigned b = 0; b < gb; ++b) t += ((u128)hp[2 * b + 1] << 64) | hp[2 * b];
    t >>= 1;  // every edge is stored twice with the same weight (odd halves only if unvalidated)
    total_w = std::ldexp((double)(u64)(t >> 64), 9) + std::ldexp((double)(u64)t, -55);  // t / 2^55
  }
  cq_graph* g = new (std::nothrow) cq_graph();
  if (!g) return fail(ctx, CQ_E_DEVICE, "out of host memory");
  g->ctx = ctx;
  g->n = n;
  g->nnz = nnz;
  g->rp = d_row_ptr;
  g->col = d_col_idx;
  g->max_degree = res[1];
  for (int b = 0; b < DEG_BINS; ++b) g->degree_bins[b] = res[2 + b];
  g->validated = validated;
  g->w = d_weights;
  g->total_w = total_w;
  if ((flags & CQ_GRAPH_REORDER) && nnz > 0) {
    const bool blocks = (flags & CQ_GRAPH_BLOCKS) ? n <= BLOCK_MAX_N
                        : !(flags & CQ_GRAPH_NO_BLOCKS) && n >= BLOCK_MIN_N && n <= BLOCK_MAX_N;
    cq_status st = build_locality_order(ctx, g, d_row_ptr, d_col_idx, blocks);
    if (st != CQ_OK) {
      delete g;
      return st;
    }
  }
  *out = g;
  return CQ_OK;
}
}  // namespace

cq_status cq_graph_load(cq_context* ctx, int32_t n, int64_t nnz, const int32_t* d_row_ptr, const int32_t* d_col_idx,
                        uint32_t flags, cq_graph** out) {
  return graph_load(ctx, n, nnz, d_row_ptr, d_col_idx, nullptr, flags, out);
}

cq_status cq_graph_load_weighted(cq_context* ctx, int32_t n, int64_t nnz, const int32_t* d_row_ptr,
                                 const int32_t* d_col_idx, const float* d_weights, uint32_t flags, cq_graph** out) {
  if (ctx && nnz > 0 && !d_weights) {
    ctx->err[0] = 0;
    return fail(ctx, CQ_E_INVALID_ARG, "null weights");
  }
  return graph_load(ctx, n, nnz, d_row_ptr, d_col_idx, nnz > 0 ? d_weights : nullptr, flags, out);
}

cq_status cq_graph_copy_order(cq_context* ctx, const cq_graph* g, int32_t* d_order) {
  if (!ctx) return CQ_E_INVALID_ARG;
  ctx->err[0] = 0;
  if (!g || !d_order) return fail(ctx, CQ_E_INVALID_ARG, "null graph or order array");
  if (!g->perm) return fail(ctx, CQ_E_INVALID_ARG, "graph was loaded without CQ_GRAPH_REORDER");
  const hipError_t e = hipMemcpyAsync(d_order, g->perm, 4 * (size_t)g->n, hipMemcpyDeviceToDevice, ctx->stream);
  if (e != hipSuccess) return fail(ctx, CQ_E_DEVICE, "copying the order: %s", hipGetErrorString(e));
  return CQ_OK;
}

cq_status cq_graph_get_stats(const cq_graph* g, cq_graph_stats* out) {
  if (!g || !out) return CQ_E_INVALID_ARG;
  out->n = g->n;
  out->nnz = g->nnz;
  out->m = g->nnz / 2;
  out->max_degree = g->max_degree;
  for (int b = 0; b < DEG_BINS; ++b) out->degree_bins[b] = g->degree_bins[b];
  out->validated = g->validated;
  out->reordered = g->reordered;
  out->weighted = g->w ? 1u : 0u;
  out->pad = 0;
  out->total_weight = g->w ? g->total_w : (double)(g->nnz / 2);
  out->clusters = g->reordered ? g->clusters : 0;
  out->largest_cluster = g->reordered ? g->largest_cluster : 0;
  out->owned_bytes = g->owned_bytes;
  return CQ_OK;
}

void cq_graph_release(cq_graph* g) { delete g; }

size_t cq_score_workspace_size(const cq_graph* g, int32_t num_labels) {
  if (!g || num_labels < 1) return 0;
  return graph_score_layout(g, num_labels).total;
}

size_t cq_compare_workspace_size(int32_t n, int32_t num_labels_a, int32_t num_labels_b) {
  if (n < 2 || num_labels_a < 1 || num_labels_b < 1) return 0;
  return cmp_layout(n, num_labels_a, num_labels_b).total;
}

cq_status cq_score_partition_async(cq_context* ctx, const cq_graph* g, const int32_t* d_labels, int32_t num_labels, void* d_ws,
                                   size_t ws_bytes, cq_score_result* d_out, const cq_per_community* per_comm,
                                   const cq_pair_table* pairs) {
  return score_enqueue(ctx, g, d_labels, num_labels, d_ws, ws_bytes, reinterpret_cast<ScoreResultDev*>(d_out), per_comm, pairs,
                       false);
}

cq_status cq_score_partition(cq_context* ctx, const cq_graph* g, const int32_t* d_labels, int32_t num_labels, void* d_ws,
                             size_t ws_bytes, cq_score_result* h_out, const cq_per_community* per_comm,
                             const cq_pair_table* pairs) {
  if (!ctx) return CQ_E_INVALID_ARG;
  if (!h_out) return fail(ctx, CQ_E_INVALID_ARG, "null result pointer");
  if (!g) return fail(ctx, CQ_E_INVALID_ARG, "null graph");
  const ScoreLayout lay = graph_score_layout(g, std::max(num_labels, 1));
  ScoreResultDev* d_res = (d_ws && ws_bytes >= lay.total) ? at<ScoreResultDev>(d_ws, lay.res) : nullptr;
  cq_status st = score_enqueue(ctx, g, d_labels, num_labels, d_ws, ws_bytes, d_res ? d_res : reinterpret_cast<ScoreResultDev*>(1),
                               per_comm, pairs, true);
  if (st != CQ_OK) return st;
  st = fetch(ctx, d_res, h_out);
  if (st != CQ_OK) return st;
  return map_flags(ctx, h_out->device_flags);
}

cq_status cq_score_partition_noalloc(cq_context* ctx, const cq_graph* g, const int32_t* d_labels, int32_t num_labels,
                                     cq_score_result* h_out, const cq_per_community* per_comm, const cq_pair_table* pairs) {
  if (!ctx) return CQ_E_INVALID_ARG;
  ctx->err[0] = 0;
  if (!h_out || !g) return fail(ctx, CQ_E_INVALID_ARG, "null graph or result pointer");
  if (!ctx->scratch) return fail(ctx, CQ_E_DEVICE, "the scratch array's address on device %d is unknown", ctx->device);
  const size_t need = graph_score_layout(g, std::max(num_labels, 1)).total;
  if (need > SCRATCH_BYTES)
    return fail(ctx, CQ_E_WORKSPACE, "this call needs %zu bytes of scratch; the library's array holds %zu "
                "(score with a caller workspace instead)", need, SCRATCH_BYTES);
  // the kernels clear what they need at the start of every call, as with a caller workspace
  return cq_score_partition(ctx, g, d_labels, num_labels, ctx->scratch, SCRATCH_BYTES, h_out, per_comm, pairs);
}

cq_status cq_compare_partitions_async(cq_context* ctx, int32_t n, const int32_t* d_labels_a, int32_t num_labels_a,
                                      const int32_t* d_labels_b, int32_t num_labels_b, void* d_ws, size_t ws_bytes,
                                      cq_compare_result* d_out, const cq_cell_table* cells) {
  return compare_enqueue(ctx, n, d_labels_a, num_labels_a, d_labels_b, num_labels_b, d_ws, ws_bytes,
                         reinterpret_cast<CmpResultDev*>(d_out), cells, false);
}

cq_status cq_compare_partitions(cq_context* ctx, int32_t n, const int32_t* d_labels_a, int32_t num_labels_a,
                                const int32_t* d_labels_b, int32_t num_labels_b, void* d_ws, size_t ws_bytes,
                                cq_compare_result* h_out, const cq_cell_table* cells) {
  if (!ctx) return CQ_E_INVALID_ARG;
  if (!h_out) return fail(ctx, CQ_E_INVALID_ARG, "null result pointer");
  const CmpLayout lay = cmp_layout(std::max(n, 2), std::max(num_labels_a, 1), std::max(num_labels_b, 1));
  CmpResultDev* d_res = (d_ws && ws_bytes >= lay.total) ? at<CmpResultDev>(d_ws, lay.res) : nullptr;
  cq_status st = compare_enqueue(ctx, n, d_labels_a, num_labels_a, d_labels_b, num_labels_b, d_ws, ws_bytes,
                                 d_res ? d_res : reinterpret_cast<CmpResultDev*>(1), cells, true);
  if (st != CQ_OK) return st;
  st = fetch(ctx, d_res, h_out);
  if (st != CQ_OK) return st;
  return map_flags(ctx, h_out->device_flags);
}

// ---- batched scoring ---------------------------------------------------------

cq_status cq_batch_plan_create(cq_context* ctx, const cq_batch_task* tasks, int32_t num_tasks, uint32_t flags,
                               cq_batch_plan** out) {
  if (!ctx) return CQ_E_INVALID_ARG;
  ctx->err[0] = 0;
  if (!out || !tasks || num_tasks < 1) return fail(ctx, CQ_E_INVALID_ARG, "null tasks or num_tasks < 1");
  *out = nullptr;
  if (flags & ~(CQ_BATCH_AUTOTUNE | CQ_BATCH_NO_GRAPH)) return fail(ctx, CQ_E_INVALID_ARG, "unknown flag bits");
  for (int i = 0; i < num_tasks; ++i) {
    const cq_batch_task& t = tasks[i];
    if (!t.graph || !t.d_labels) return fail(ctx, CQ_E_INVALID_ARG, "task %d: null graph or labels", i);
    if (t.graph->w) return fail(ctx, CQ_E_INVALID_ARG, "task %d: weighted graphs are scored one call at a time", i);
    if (t.num_labels < 1 || t.num_labels > BATCH_MAX_L)
      return fail(ctx, CQ_E_INVALID_ARG, "task %d: num_labels must be in [1, %lld] for batching", i, (long long)BATCH_MAX_L);
    if (t.graph->nnz == 0) return fail(ctx, CQ_E_NO_EDGES, "task %d: graph has no edges", i);
  }
  if (num_tasks > BATCH_MAX_TASKS) return fail(ctx, CQ_E_INVALID_ARG, "at most %d tasks per batch", BATCH_MAX_TASKS);
  cq_batch_plan* p = new (std::nothrow) cq_batch_plan();
  if (!p) return fail(ctx, CQ_E_DEVICE, "out of host memory");
  p->ctx = ctx;
  p->flags = flags;
  p->tasks.assign(tasks, tasks + num_tasks);
  batch_layout(p);
  if (hipStreamCreateWithFlags(&p->stream, hipStreamNonBlocking) != hipSuccess ||
      hipEventCreateWithFlags(&p->ev_in, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&p->ev_out, hipEventDisableTiming) != hipSuccess ||
      hipHostMalloc(&p->pinned, sizeof(cq_score_result) * (size_t)num_tasks, hipHostMallocDefault) != hipSuccess) {
    delete p;
    return fail(ctx, CQ_E_DEVICE, "creating batch stream/events");
  }
  *out = p;
  return CQ_OK;
}

size_t cq_batch_workspace_size(const cq_batch_plan* p) { return p ? p->ws_total : 0; }

cq_status cq_batch_bind(cq_batch_plan* p, void* d_ws, size_t ws_bytes, cq_score_result* d_results) {
  if (!p) return CQ_E_INVALID_ARG;
  cq_context* ctx = p->ctx;
  ctx->err[0] = 0;
  if (!d_ws || ws_bytes < p->ws_total)
    return fail(ctx, CQ_E_WORKSPACE, "workspace %zu bytes, need %zu", ws_bytes, p->ws_total);
  if (reinterpret_cast<uintptr_t>(d_ws) % WS_ALIGN) return fail(ctx, CQ_E_INVALID_ARG, "workspace not 16-byte aligned");
  if (!d_results) return fail(ctx, CQ_E_INVALID_ARG, "null result array");
  if (p->exec) { (void)hipGraphExecDestroy(p->exec); p->exec = nullptr; }
  if (p->graph) { (void)hipGraphDestroy(p->graph); p->graph = nullptr; }
  if (p->d_tab) { (void)hipFree(p->d_tab); p->d_tab = nullptr; }
  p->bound = false;
  const BatchTabLayout tl = batch_tab_layout((int)p->tasks.size(), (int)p->groups.size());
  if (hipMalloc(&p->d_tab, tl.total) != hipSuccess) return fail(ctx, CQ_E_DEVICE, "allocating batch tables");
  p->tab_bytes = tl.total;
  std::vector<char> blob(tl.total);
  batch_fill_tables(p, d_ws, d_results, blob.data(), p->d_tab);
  hipStream_t s = p->stream;
  hipError_t e = hipMemcpyAsync(p->d_tab, blob.data(), tl.total, hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return fail(ctx, CQ_E_DEVICE, "uploading batch tables: %s", hipGetErrorString(e));

  // choose the tiling: cached choice, or time every candidate on this batch
  const int maxocc = batch_max_occ(p);
  p->rsel = 1;
  p->occ = maxocc;
  p->tuned_ms = 0.0;
  p->from_cache = 0;
  if (p->flags & CQ_BATCH_AUTOTUNE) {
    const std::string key = batch_key(p);
    int rs = 1, oc = maxocc;
    double ms = 0.0;
    if (tune_lookup(key, &rs, &oc, &ms) && oc <= maxocc) {
      p->rsel = rs;
      p->occ = oc;
      p->tuned_ms = ms;
      p->from_cache = 1;
    } else {
      hipEvent_t a, z;
      (void)hipEventCreate(&a);
      (void)hipEventCreate(&z);
      double best = 1e30;
      std::vector<int> occs = {1, 2, maxocc};
      for (int r = 0; r < 3; ++r) {
        for (int oc2 : occs) {
          if (oc2 > maxocc) continue;
          batch_launch(p, s, r, oc2);  // warm
          (void)hipEventRecord(a, s);
          batch_launch(p, s, r, oc2);
          (void)hipEventRecord(z, s);
          (void)hipEventSynchronize(z);
          float t = 0.f;
          (void)hipEventElapsedTime(&t, a, z);
          if (t < best) {
            best = t;
            p->rsel = r;
            p->occ = oc2;
          }
        }
      }
      (void)hipEventDestroy(a);
      (void)hipEventDestroy(z);
      p->tuned_ms = best;
      tune_store(key, p->rsel, p->occ, best);
    }
  }
  e = hipGetLastError();
  if (e != hipSuccess) return fail(ctx, CQ_E_DEVICE, "batch tuning: %s", hipGetErrorString(e));
  p->graph_nodes = 0;
  if (!(p->flags & CQ_BATCH_NO_GRAPH)) {
    e = hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
      batch_launch(p, s, p->rsel, p->occ);
      e = hipStreamEndCapture(s, &p->graph);
    }
    if (e == hipSuccess) e = hipGraphInstantiate(&p->exec, p->graph, nullptr, nullptr, 0);
    if (e != hipSuccess) return fail(ctx, CQ_E_DEVICE, "capturing the batch graph: %s", hipGetErrorString(e));
    size_t nn = 0;
    if (hipGraphGetNodes(p->graph, nullptr, &nn) == hipSuccess) p->graph_nodes = (int)nn;
  }
  p->bound = true;
  return CQ_OK;
}

cq_status cq_batch_run(cq_batch_plan* p) {
  if (!p) return CQ_E_INVALID_ARG;
  cq_context* ctx = p->ctx;
  if (!p->bound) return fail(ctx, CQ_E_INVALID_ARG, "batch plan is not bound");
  hipError_t e = hipEventRecord(p->ev_in, ctx->stream);
  if (e == hipSuccess) e = hipStreamWaitEvent(p->stream, p->ev_in, 0);
  if (e == hipSuccess) {
    if (p->exec) e = hipGraphLaunch(p->exec, p->stream);
    else {
      batch_launch(p, p->stream, p->rsel, p->occ);
      e = hipGetLastError();
    }
  }
  if (e == hipSuccess) e = hipEventRecord(p->ev_out, p->stream);
  if (e == hipSuccess) e = hipStreamWaitEvent(ctx->stream, p->ev_out, 0);
  if (e != hipSuccess) return fail(ctx, CQ_E_DEVICE, "batch run: %s", hipGetErrorString(e));
  return CQ_OK;
}

cq_status cq_batch_run_sync(cq_batch_plan* p, cq_score_result* h_results) {
  if (!p) return CQ_E_INVALID_ARG;
  cq_context* ctx = p->ctx;
  if (!h_results) return fail(ctx, CQ_E_INVALID_ARG, "null host result array");
  cq_status st = cq_batch_run(p);
  if (st != CQ_OK) return st;
  const size_t bytes = sizeof(cq_score_result) * p->tasks.size();
  hipError_t e = hipMemcpyAsync(p->pinned, p->d_results, bytes, hipMemcpyDeviceToHost, ctx->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
  if (e != hipSuccess) return fail(ctx, CQ_E_DEVICE, "batch results: %s", hipGetErrorString(e));
  std::memcpy(h_results, p->pinned, bytes);
  for (size_t t = 0; t < p->tasks.size(); ++t) {
    if (h_results[t].device_flags) {
      cq_status fs = map_flags(ctx, h_results[t].device_flags);
      char msg[64];
      snprintf(msg, sizeof(msg), " (task %zu)", t);
      strncat(ctx->err, msg, sizeof(ctx->err) - strlen(ctx->err) - 1);
      return fs;
    }
  }
  return CQ_OK;
}

cq_status cq_batch_get_tuning(const cq_batch_plan* p, cq_batch_tuning* out) {
  if (!p || !out) return CQ_E_INVALID_ARG;
  out->gather_rows = kGatherRows[p->rsel];
  out->group_blocks_per_cu = p->occ;
  out->tuned_ms = p->tuned_ms;
  out->from_cache = p->from_cache;
  out->graph_nodes = p->graph_nodes;
  out->num_groups = (int32_t)p->groups.size();
  return CQ_OK;
}

void cq_batch_plan_destroy(cq_batch_plan* p) { delete p; }

// ---- serving -------------------------------------------------------------------

cq_status cq_server_create(cq_context* ctx, const cq_server_config* cfg, cq_server** out) {
  if (!ctx) return CQ_E_INVALID_ARG;
  ctx->err[0] = 0;
  if (!cfg || !out) return fail(ctx, CQ_E_INVALID_ARG, "null config or output");
  *out = nullptr;
  if (cfg->num_slots < 1 || cfg->num_slots > 64 || cfg->max_batch < 1 || cfg->max_batch > 4096 || cfg->memory_budget < 4096)
    return fail(ctx, CQ_E_INVALID_ARG, "num_slots in [1, 64], max_batch in [1, 4096], memory_budget >= 4096");
  cq_server* s = new (std::nothrow) cq_server();
  if (!s) return fail(ctx, CQ_E_DEVICE, "out of host memory");
  s->ctx = ctx;
  s->cfg = *cfg;
  s->exec.device = ctx->device;
  hipError_t e = hipMalloc((void**)&s->exec.arena, (size_t)cfg->memory_budget);
  if (e != hipSuccess) {
    delete s;
    return fail(ctx, CQ_E_DEVICE, "allocating the server arena: %s", hipGetErrorString(e));
  }
  const BatchTabLayout tl = batch_tab_layout(cfg->max_batch, cfg->max_batch);
  const size_t res_bytes = aup(std::max(sizeof(cq_compare_result), sizeof(cq_score_result) * (size_t)cfg->max_batch));
  for (int i = 0; i < cfg->num_slots && e == hipSuccess; ++i) {
    SrvSlot* sl = new SrvSlot();
    s->exec.slots.push_back(sl);
    e = hipStreamCreateWithFlags(&sl->stream, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&sl->ev, hipEventDisableTiming);
    if (e == hipSuccess) e = hipHostMalloc((void**)&sl->pinned, res_bytes + tl.total, hipHostMallocDefault);
    if (e == hipSuccess) e = hipMalloc(&sl->d_tab, tl.total);
    if (e == hipSuccess && cq_context_create(ctx->device, sl->stream, &sl->ctx) != CQ_OK) e = hipErrorUnknown;
    sl->res_bytes = res_bytes;
    sl->plan.ctx = sl->ctx;
  }
  if (e != hipSuccess) {
    cq_server_destroy(s);
    return fail(ctx, CQ_E_DEVICE, "creating server slots: %s", hipGetErrorString(e));
  }
  cqsrv::Config sc;
  sc.num_slots = cfg->num_slots;
  sc.max_batch = cfg->max_batch;
  sc.arena_bytes = (size_t)cfg->memory_budget;
  s->sched = new (std::nothrow) cqsrv::Scheduler(sc, &s->exec);
  if (!s->sched) {
    cq_server_destroy(s);
    return fail(ctx, CQ_E_DEVICE, "out of host memory");
  }
  s->sched->start();
  *out = s;
  return CQ_OK;
}

cq_status cq_server_submit_score(cq_server* srv, const cq_graph* g, const int32_t* h_labels, int32_t num_labels,
                                 uint64_t* ticket) {
  if (!srv) return CQ_E_INVALID_ARG;
  if (!g || !h_labels || !ticket || num_labels < 1) return fail(srv->ctx, CQ_E_INVALID_ARG, "bad scoring request");
  if (g->nnz == 0) return fail(srv->ctx, CQ_E_NO_EDGES, "graph has no edges");
  cqsrv::Req* r = new (std::nothrow) cqsrv::Req();
  if (!r) return CQ_E_DEVICE;
  r->kind = 0;
  r->graph = g;
  r->n = g->n;
  r->L = num_labels;
  r->ha = h_labels;
  r->ws_bytes = graph_score_layout(g, num_labels).total;
  // inside a grouped launch: the task's workspace and, at most, one group's interleaved
  // labels (8 bytes per node; batch_layout)
  r->group_ws = cqsrv::aup(score_layout(g->n, g->nnz, num_labels).total) + cqsrv::aup(8 * (size_t)g->n);
  r->small = num_labels <= BATCH_MAX_L && g->nnz <= srv->cfg.small_nnz && !g->w;  // groups run the unweighted batch kernels
  return srv_submit(srv, r, ticket);
}

cq_status cq_server_submit_compare(cq_server* srv, int32_t n, const int32_t* h_labels_a, int32_t num_labels_a,
                                   const int32_t* h_labels_b, int32_t num_labels_b, uint64_t* ticket) {
  if (!srv) return CQ_E_INVALID_ARG;
  if (n < 2 || !h_labels_a || !h_labels_b || !ticket || num_labels_a < 1 || num_labels_b < 1)
    return fail(srv->ctx, CQ_E_INVALID_ARG, "bad comparison request");
  cqsrv::Req* r = new (std::nothrow) cqsrv::Req();
  if (!r) return CQ_E_DEVICE;
  r->kind = 1;
  r->n = n;
  r->La = num_labels_a;
  r->Lb = num_labels_b;
  r->ha = h_labels_a;
  r->hb = h_labels_b;
  r->ws_bytes = cmp_layout(n, num_labels_a, num_labels_b).total;
  return srv_submit(srv, r, ticket);
}

cq_status cq_server_wait(cq_server* srv, uint64_t ticket, double timeout_ms, cq_status* request_status,
                         cq_score_result* score_out, cq_compare_result* compare_out, double* latency_ms) {
  if (!srv) return CQ_E_INVALID_ARG;
  cqsrv::Outcome o;
  const char* why = nullptr;
  const cq_status st = srv->sched->wait(ticket, timeout_ms, &o, &why);
  if (st == CQ_E_INVALID_ARG) return fail(srv->ctx, st, "%s", why ? why : "bad ticket");
  if (st != CQ_OK) return st;
  if (request_status) *request_status = o.status;
  if (score_out && o.kind == 0) *score_out = o.sres;
  if (compare_out && o.kind == 1) *compare_out = o.cres;
  if (latency_ms) *latency_ms = o.latency_ms;
  return CQ_OK;
}

cq_status cq_server_get_stats(cq_server* srv, cq_server_stats* out) {
  if (!srv || !out) return CQ_E_INVALID_ARG;
  srv->sched->stats(out);
  return CQ_OK;
}

cq_status cq_server_reset_stats(cq_server* srv) {
  if (!srv) return CQ_E_INVALID_ARG;
  srv->sched->reset_stats();
  return CQ_OK;
}

void cq_server_destroy(cq_server* srv) {
  if (!srv) return;
  // cancels what is queued, lets the admitted work finish, and returns once no thread
  // is left inside cq_server_wait
  if (srv->sched) srv->sched->shutdown();
  for (SrvSlot* sl : srv->exec.slots) {
    if (sl->stream) (void)hipStreamSynchronize(sl->stream);
    if (sl->ctx) cq_context_destroy(sl->ctx);
    if (sl->ev) (void)hipEventDestroy(sl->ev);
    if (sl->stream) (void)hipStreamDestroy(sl->stream);
    if (sl->pinned) (void)hipHostFree(sl->pinned);
    if (sl->d_tab) (void)hipFree(sl->d_tab);
    sl->plan.stream = nullptr;  // the plan object owns nothing here
    delete sl;
  }
  srv->exec.slots.clear();
  delete srv->sched;
  if (srv->exec.arena) (void)hipFree(srv->exec.arena);
  delete srv;
}

}  // extern "C"
