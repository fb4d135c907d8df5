/*
 * cq.h -- C ABI of the MI355X (gfx950) community-quality library.
 *
 * Computes the community-quality metrics of Chen, Liu and Szymanski, "Parallel
 * Toolkit for Measuring the Quality of Network Community Structure":
 *   - scoring one partition of an unweighted undirected graph (Section II-B):
 *     modularity Q (Eq. 8), modularity density Qds (Eq. 9), and the six measures
 *     of Section II-B3 (intra-edges, intra-density, contraction, inter-edges,
 *     expansion, conductance);
 *   - comparing a ground-truth partition C with a detected partition C'
 *     (Section II-A): VI (Eq. 1), NMI (Eq. 2), F-measure (Eq. 3), NVD (Eq. 4),
 *     RI (Eq. 5), ARI (Eq. 6), JI (Eq. 7) and the pair counts of Section II-A3.
 *
 * Conventions shared by every entry point
 *   Memory     All arrays marked DEVICE are device pointers owned by the caller
 *              (for example the storage of torch tensors).  The library never
 *              frees caller memory and never allocates device memory inside a
 *              scoring or comparison call; scratch space is the caller-provided
 *              workspace, sized by the *_workspace_size queries and 16-byte aligned
 *              (hipMalloc's alignment is enough).  Structs marked HOST are host memory.
 *   Streams    Work is enqueued on the context's HIP stream (hipStream_t passed
 *              as void*).  Synchronous calls return after the result struct has
 *              reached host memory.
 *   Errors     Every call returns a cq_status.  Argument errors detectable on the
 *              host return before anything is enqueued.  Errors found by the
 *              kernels (a label outside [0, num_labels)) are reported through a
 *              device flag word and mapped to CQ_E_LABEL_RANGE; the numeric
 *              outputs of that call are then unspecified.  cq_context_last_error()
 *              gives a one-line description of the last failure on a context.
 *   Threads    A context and everything enqueued through it belong to one host
 *              thread at a time.
 *   Sizes      Graphs use int32 CSR (row offsets and column indices), so the
 *              number of stored entries 2|E| must be below 2^31.  All counts the
 *              library returns are exact integers; floating-point outputs are
 *              binary64.
 */
#ifndef CQ_H
#define CQ_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t cq_status;
#define CQ_OK 0
#define CQ_E_INVALID_ARG (-1)   /* null pointer, bad size, bad flag */
#define CQ_E_LABEL_RANGE (-2)   /* a label outside [0, num_labels) */
#define CQ_E_GRAPH_FORMAT (-3)  /* CSR not well formed, or (when validated) not symmetric / has loops / duplicates */
#define CQ_E_OVERFLOW (-4)      /* a size exceeds the int32 CSR limits */
#define CQ_E_WORKSPACE (-5)     /* workspace missing or smaller than the size query returned */
#define CQ_E_NO_EDGES (-6)      /* graph has no edges: Q and Qds divide by |E| */
#define CQ_E_DEVICE (-7)        /* a HIP runtime call failed */
#define CQ_E_BUSY (-8)          /* server: request not admitted */
#define CQ_E_CANCELLED (-9)     /* server: request cancelled */
#define CQ_E_CAPACITY (-10)     /* an optional export table was too small; all other outputs are valid */

/* Human-readable name of a status code (static storage). */
const char* cq_status_string(cq_status s);

typedef struct cq_context cq_context;
typedef struct cq_graph cq_graph;

/* Create a context bound to HIP device `device`, enqueueing on `hip_stream`
 * (a hipStream_t; NULL means the default stream).  *out receives the handle. */
cq_status cq_context_create(int device, void* hip_stream, cq_context** out);
/* Change the stream later calls enqueue on. */
cq_status cq_context_set_stream(cq_context* ctx, void* hip_stream);
void cq_context_destroy(cq_context* ctx);
/* One-line description of the last failing call on ctx ("" if none). */
const char* cq_context_last_error(const cq_context* ctx);

/* ---- stage timing (tracing) ------------------------------------------------ */

/* When timing is enabled on a context, every stage of a synchronous call
 * (cq_score_partition, cq_compare_partitions) is bracketed by HIP events recorded on
 * the context's stream; after the call synchronises, each stage's elapsed time is
 * added to a per-stage total.  Stage ids are small integers named by cq_stage_name.
 * Asynchronous calls are not timed. */
#define CQ_MAX_STAGES 12
/* enable != 0 turns timing on for every stage, 0 off; both reset the totals. */
cq_status cq_context_enable_timing(cq_context* ctx, int enable);
/* Time only the stages whose bit (1 << stage id) is set in stage_mask (0: off); resets
 * the totals.  Each timed stage adds two event records to the stream, which cost a few
 * microseconds of device time, so a caller that needs one stage's duration times that
 * stage alone. */
cq_status cq_context_time_stages(cq_context* ctx, uint32_t stage_mask);
/* Copy up to max_stages per-stage totals (milliseconds) and counts (timed calls
 * that ran the stage) into the HOST arrays total_ms[] and counts[]. */
cq_status cq_context_stage_times(const cq_context* ctx, double* total_ms, int64_t* counts, int32_t max_stages);
/* Name of stage id s (static storage), or "" if s is not a stage id. */
const char* cq_stage_name(int32_t s);

/* ---- staging choice on column-blocked graphs -------------------------------- */

/* A column-blocked graph stores nodes so that communities found at load time are runs of
 * consecutive ids, and stages neighbour labels with one claim per run of equal labels.  A
 * partition that does not follow that order (say, a perturbed or unrelated one) breaks
 * the runs, and the claims grow to one per node.  Each unweighted call on such a graph
 * (with up to 12,224 label ids) therefore counts, on the device, the label changes between
 * consecutive stored nodes; when they reach change_fraction * n the call stages through
 * the graph's row-major copy with per-node offsets instead (cq_score_result.staging says
 * which).  Default 1/16; <= 0 always takes the row-major copy, >= 1 never does.  The
 * results are the same either way. */
cq_status cq_context_set_row_staging(cq_context* ctx, double change_fraction);

/* ---- graphs ---------------------------------------------------------------- */

/* Flags for cq_graph_load. */
#define CQ_VALIDATE_GRAPH 1u  /* also check symmetry (rows must be sorted), no self-loops, no repeated entries */
#define CQ_GRAPH_REORDER 2u   /* store the graph in a locality order (see cq_graph_load) */
#define CQ_GRAPH_NO_BLOCKS 4u /* with CQ_GRAPH_REORDER: never build column blocks (see cq_graph_load) */
#define CQ_GRAPH_BLOCKS 8u    /* with CQ_GRAPH_REORDER: build column blocks for any n <= 2^24 */

typedef struct {
  int64_t n;           /* |V| */
  int64_t nnz;         /* stored CSR entries = 2|E| */
  int64_t m;           /* |E| */
  int64_t max_degree;
  uint32_t validated;  /* CQ_VALIDATE_GRAPH if the full check ran and passed */
  uint32_t reordered;  /* CQ_GRAPH_REORDER if the graph is stored in a locality order, plus
                          CQ_GRAPH_NO_BLOCKS if it is stored without column blocks */
  int64_t owned_bytes; /* device memory the graph handle allocated (0 without CQ_GRAPH_REORDER) */
  uint32_t weighted;   /* 1 for a graph registered with cq_graph_load_weighted */
  uint32_t pad;
  double total_weight; /* W: sum of the edge weights (|E| for an unweighted graph) */
  int64_t clusters;        /* CQ_GRAPH_REORDER: label-propagation clusters the order groups (else 0) */
  int64_t largest_cluster; /* nodes in the largest of them (else 0) */
  int64_t degree_bins[32]; /* nodes per degree bin: [0] degree 0, [b] degrees in [2^(b-1), 2^b) */
} cq_graph_stats;

/*
 * Register a graph: the symmetric CSR of a simple unweighted undirected graph
 * G = (V, E) (Section II-B1), with every undirected edge stored in both rows.
 *   n          number of nodes, >= 1
 *   nnz        number of stored entries, row_ptr[n]; even, < 2^31
 *   d_row_ptr  DEVICE int32[n+1], row_ptr[0] = 0, non-decreasing, row_ptr[n] = nnz
 *   d_col_idx  DEVICE int32[nnz], entries in [0, n)
 * The pointers are BORROWED: the arrays must stay alive and unchanged until
 * cq_graph_release.  The structural checks above always run (one pass over the
 * arrays, synchronous); CQ_VALIDATE_GRAPH adds the symmetry / loop / repeat checks.
 * Returns CQ_E_GRAPH_FORMAT if a check fails.
 * CQ_GRAPH_REORDER: the handle builds and owns a renumbered copy of the graph
 * (4(n+1) + 4 nnz + 4n bytes of device memory, allocated here and freed by
 * cq_graph_release) in which nodes are grouped by a few sweeps of label propagation,
 * so that the neighbours of a row mostly have nearby ids.  Labels passed to scoring
 * calls keep the caller's node numbering; every result is identical with and without
 * the flag.  The borrowed arrays are not read after the load returns.
 * When 2^20 <= n <= 2^24 the copy is also kept as 8 column blocks, one per XCD of the
 * device (the edge pass then reads each neighbour label from one XCD's L2; below 2^20
 * nodes one L2 holds all labels anyway), with a plan that moves labels from the
 * caller's order to the stored one: a further 4(8(n+1)+1) + 8 nnz + 16n + 4(n/32768 + 2)
 * bytes.  CQ_GRAPH_NO_BLOCKS never builds them, CQ_GRAPH_BLOCKS builds them for any
 * n <= 2^24 (both flags at once: CQ_E_INVALID_ARG).  owned_bytes in cq_graph_stats
 * reports the total.
 */
cq_status cq_graph_load(cq_context* ctx, int32_t n, int64_t nnz, const int32_t* d_row_ptr,
                        const int32_t* d_col_idx, uint32_t flags, cq_graph** out);
/*
 * Register an edge-weighted graph: as cq_graph_load, plus
 *   d_weights  DEVICE float[nnz], the weight of every stored entry, BORROWED like the
 *              CSR arrays; finite, in [2^-32, 2^32], and equal for the two entries of
 *              an undirected edge.  A weighted load always runs the CQ_VALIDATE_GRAPH
 *              checks (rows sorted, symmetric, simple) together with that equality.
 * Scoring a weighted graph gives Eqs. 8-9 and the measures of Section II-B3 with
 * weight sums in place of edge counts, while the densities d_c and d_{ci,cj} keep the
 * unweighted counts (the paper's note for weighted networks): see cq_score_result.
 * The total weight is summed exactly at load (cq_graph_stats.total_weight).
 * Returns CQ_E_GRAPH_FORMAT for a weight outside the range or a mismatched pair.
 */
cq_status cq_graph_load_weighted(cq_context* ctx, int32_t n, int64_t nnz, const int32_t* d_row_ptr,
                                 const int32_t* d_col_idx, const float* d_weights, uint32_t flags,
                                 cq_graph** out);
cq_status cq_graph_get_stats(const cq_graph* g, cq_graph_stats* out);
/* Copy the stored node order of a graph loaded with CQ_GRAPH_REORDER into the DEVICE
 * array d_order[n]: d_order[i] is the caller's id of the i-th stored node.  Enqueued on
 * the context's stream (asynchronous).  CQ_E_INVALID_ARG if the graph was not
 * renumbered or d_order is null. */
cq_status cq_graph_copy_order(cq_context* ctx, const cq_graph* g, int32_t* d_order);
void cq_graph_release(cq_graph* g);

/* ---- scoring one partition (Section II-B) ---------------------------------- */

/* HOST result of cq_score_partition.  "Communities" are the label ids carried by
 * at least one node; K counts them; means are unweighted over those K.
 * Weighted graphs (weighted = 1): the integer fields keep the unweighted edge counts;
 * Q, Qds, split_penalty and the means of intra-edges (w_in), contraction (2 w_in/|c|),
 * inter-edges (w_out), expansion (w_out/|c|) and conductance (w_out/s(c)) use weight
 * sums, with W = total_weight in place of |E| and s(c) = 2 w_in(c) + w_out(c); the
 * intra-density mean and the pair densities inside Qds use the unweighted counts. */
typedef struct {
  int64_t n, m;              /* |V|, |E| */
  int64_t K;                 /* non-empty communities */
  int64_t num_pairs;         /* unordered community pairs joined by at least one edge */
  int64_t sum_ein;           /* sum_c |E_c^in|  (intra-edges, Section II-B3) */
  int64_t sum_eout;          /* sum_c |E_c^out| (inter-edges, Section II-B3) */
  uint64_t sum_degsum_sq;    /* sum_c (2|E_c^in| + |E_c^out|)^2, exact */
  double Q;                  /* Eq. 8 */
  double Qds;                /* Eq. 9 */
  double split_penalty;      /* sum_i sum_{j != i} |E_ij| / (2|E|) * d_ij, the subtracted part of Eq. 9 */
  double mean_intra_edges, mean_intra_density, mean_contraction;
  double mean_inter_edges, mean_expansion, mean_conductance;
  uint32_t device_flags;     /* raw device error bits (0 on success) */
  uint32_t weighted;         /* 1 when the graph is edge-weighted */
  double total_weight;       /* W (|E| when unweighted) */
  double sum_w_in;           /* sum_c w_in(c) (sum_ein when unweighted) */
  double sum_w_out;          /* sum_c w_out(c) (sum_eout when unweighted) */
  uint32_t staging;          /* how the neighbour labels were staged: CQ_STAGING_* (informational) */
  uint32_t reserved;
} cq_score_result;

/* cq_score_result.staging.  The results do not depend on it. */
#define CQ_STAGING_ROWS_ONLY 0u  /* the graph's row-major storage (no column blocks; batched calls) */
#define CQ_STAGING_BLOCKS 1u     /* column blocks, compact staging with one claim per run of equal labels */
#define CQ_STAGING_ROWS 2u       /* a column-blocked graph staged through its row-major copy: the partition
                                    does not follow the stored order (see cq_context_set_row_staging) */

/* Optional per-label outputs: DEVICE arrays of length num_labels, each may be NULL.
 * Entries for label ids that no node carries are zero.  On a weighted graph
 * contraction, expansion, conductance, q_term and qds_term take the weight sums of
 * cq_score_result (2 w_in(c)/|c|, w_out(c)/|c|, w_out(c)/s(c)); size, degsum, ein,
 * eout and intra_density stay unweighted counts. */
typedef struct {
  int64_t* size;           /* |c| */
  int64_t* degsum;         /* 2|E_c^in| + |E_c^out| */
  int64_t* ein;            /* |E_c^in|  (intra-edges) */
  int64_t* eout;           /* |E_c^out| (inter-edges) */
  double* intra_density;   /* d_c = 2|E_c^in| / (|c|(|c|-1)); 0 when |c| < 2 */
  double* contraction;     /* 2|E_c^in| / |c| */
  double* expansion;       /* |E_c^out| / |c| */
  double* conductance;     /* |E_c^out| / (2|E_c^in| + |E_c^out|); 0 when that is 0 */
  double* q_term;          /* bracket of Eq. 8 for c */
  double* qds_term;        /* bracket of Eq. 9 for c (including its split-penalty sum) */
  double* w_in;            /* weighted graphs: w_in(c) (ignored otherwise) */
  double* strength;        /* weighted graphs: s(c) = 2 w_in(c) + w_out(c) (ignored otherwise) */
} cq_per_community;
/* (On a weighted graph contraction, expansion, conductance, q_term and qds_term are the
 * weighted forms; size, degsum, ein, eout and intra_density stay unweighted.) */

/* Optional export of the inter-community edge counts |E_{ci,cj}| (Eq. 9): DEVICE
 * arrays of `capacity` entries; one entry per unordered pair ci < cj with a
 * non-zero count, in unspecified order.  If capacity is too small the call
 * returns CQ_E_CAPACITY (all other outputs valid; result.num_pairs is exact). */
typedef struct {
  int32_t* ci;
  int32_t* cj;
  int64_t* count;
  int64_t capacity;
} cq_pair_table;

/* Bytes of workspace cq_score_partition needs for graph g and num_labels ids. */
size_t cq_score_workspace_size(const cq_graph* g, int32_t num_labels);

/*
 * Score the partition given by d_labels (DEVICE int32[n], values in
 * [0, num_labels); ids no node carries are allowed and ignored).
 *   d_ws/ws_bytes  DEVICE workspace of at least cq_score_workspace_size bytes, 16-byte
 *                  aligned (as hipMalloc returns; CQ_E_INVALID_ARG otherwise);
 *                  contents on entry are ignored, on exit unspecified.
 *   h_out          HOST result.
 *   per_comm       optional per-label DEVICE outputs (NULL to skip).
 *   pairs          optional pair-table export (NULL to skip).
 * Synchronous.  Errors: CQ_E_INVALID_ARG (also: a weighted graph with more than
 * 32768 label ids), CQ_E_WORKSPACE, CQ_E_NO_EDGES, CQ_E_LABEL_RANGE, CQ_E_CAPACITY,
 * CQ_E_DEVICE.
 */
cq_status cq_score_partition(cq_context* ctx, const cq_graph* g, const int32_t* d_labels,
                             int32_t num_labels, void* d_ws, size_t ws_bytes, cq_score_result* h_out,
                             const cq_per_community* per_comm, const cq_pair_table* pairs);

/* Asynchronous form: enqueue the same work and write the result struct to DEVICE
 * memory d_out (a cq_score_result, 8-byte aligned) without synchronising.  Host
 * argument errors are returned immediately; device-detected errors appear in
 * d_out->device_flags (bit 0: label out of range; bit 2: pair export overflow). */
cq_status cq_score_partition_async(cq_context* ctx, const cq_graph* g, const int32_t* d_labels,
                                   int32_t num_labels, void* d_ws, size_t ws_bytes,
                                   cq_score_result* d_out, const cq_per_community* per_comm,
                                   const cq_pair_table* pairs);

/* ---- scoring without a workspace (callers that cannot allocate) ------------- */

/* Bytes of the library's own scratch array (one per device). */
#define CQ_SCRATCH_BYTES (64u << 20)

/*
 * For callers that cannot allocate device memory: code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc.  Same as cq_score_partition (same
 * outputs, bit for bit), with the library's own scratch array of CQ_SCRATCH_BYTES in
 * place of the caller's workspace; the caller still provides labels and the optional
 * per_comm / pairs outputs.  The array is device memory the library holds on every GPU
 * it runs on until the process ends; its address on a device is looked up once, when
 * the first context on that device is created.  The call allocates nothing (no
 * hipMalloc, hipFree or allocating library routine) and clears what must start at zero.
 * Every call on one GPU shares that GPU's array: calls that overlap on one GPU (from
 * several contexts, threads or streams) race and give undefined results; calls on one
 * stream are ordered and safe.
 * Errors: those of cq_score_partition, plus CQ_E_WORKSPACE when the call would need more
 * than CQ_SCRATCH_BYTES (cq_score_workspace_size(g, num_labels) says how much; about
 * 2 bytes per stored entry plus a few bytes per node and per label), and CQ_E_DEVICE if
 * the array's device address could not be found.  Synchronous.
 */
cq_status cq_score_partition_noalloc(cq_context* ctx, const cq_graph* g, const int32_t* d_labels, int32_t num_labels,
                                     cq_score_result* h_out, const cq_per_community* per_comm,
                                     const cq_pair_table* pairs);

/* ---- batched scoring (many graphs x many partitions) ------------------------ */

/* A batch scores many (graph, partition) tasks with one launch per stage of the
 * scoring path instead of one call per task: every stage works on all tasks at once,
 * partitions of the same graph share one read of its col_idx (up to 4 per group), and
 * the per-community pass is one persistent launch over the communities of all tasks.
 * The stage sequence is captured once in a HIP graph and replayed by cq_batch_run.
 * Results are those of cq_score_partition for each task (bit for bit).
 * Envelope: 1 <= num_labels <= 16384 per task, unweighted graphs with at least one
 * edge; larger label spaces and weighted graphs go through cq_score_partition. */
typedef struct {
  const cq_graph* graph;    /* registered graph (may be shared by several tasks) */
  const int32_t* d_labels;  /* DEVICE int32[n], read at every run (contents may change between runs) */
  int32_t num_labels;
} cq_batch_task;

typedef struct cq_batch_plan cq_batch_plan;

#define CQ_BATCH_AUTOTUNE 1u  /* time candidate tilings on this batch at bind and keep the fastest */
#define CQ_BATCH_NO_GRAPH 2u  /* launch the stage kernels directly instead of replaying a HIP graph */

/* Validate tasks and lay out the batch (host only; copies the task array). */
cq_status cq_batch_plan_create(cq_context* ctx, const cq_batch_task* tasks, int32_t num_tasks, uint32_t flags,
                               cq_batch_plan** out);
/* Workspace bytes the plan needs (0 for a null plan). */
size_t cq_batch_workspace_size(const cq_batch_plan* plan);
/* Bind DEVICE workspace and a DEVICE result array (cq_score_result[num_tasks]) to the
 * plan: builds the device task tables (plan-owned device memory), autotunes when asked
 * (this runs the batch), and captures the HIP graph.  Rebinding replaces all of this. */
cq_status cq_batch_bind(cq_batch_plan* plan, void* d_ws, size_t ws_bytes, cq_score_result* d_results);
/* Enqueue one run of the bound batch, ordered after earlier work on the context's stream. */
cq_status cq_batch_run(cq_batch_plan* plan);
/* Run, copy all results to HOST h_results[num_tasks] and synchronise.  Returns
 * CQ_E_LABEL_RANGE if any task had a label outside its range (its results are then
 * unspecified; the others are valid). */
cq_status cq_batch_run_sync(cq_batch_plan* plan, cq_score_result* h_results);

typedef struct {
  int32_t gather_rows;          /* rows per workgroup of the batched edge pass */
  int32_t group_blocks_per_cu;  /* resident workgroups per CU of the persistent group pass */
  double tuned_ms;              /* fastest candidate's time (0 if not autotuned) */
  int32_t from_cache;           /* 1 if the choice came from the tuning cache */
  int32_t graph_nodes;          /* nodes of the captured HIP graph (0 with CQ_BATCH_NO_GRAPH) */
  int32_t num_groups;           /* graph groups (partitions sharing one graph read) */
} cq_batch_tuning;
cq_status cq_batch_get_tuning(const cq_batch_plan* plan, cq_batch_tuning* out);
void cq_batch_plan_destroy(cq_batch_plan* plan);

/* ---- comparing two partitions (Section II-A) -------------------------------- */

/* HOST result of cq_compare_partitions.  C is the ground truth (labels a), C' the
 * detected partition (labels b).  Pair counts are over unordered node pairs. */
typedef struct {
  int64_t n;                 /* |V| */
  int64_t Ka, Kb;            /* non-empty communities of C and C' */
  int64_t nnz;               /* non-zero cells |c ∩ c'| of the contingency table */
  int64_t a11, a10, a01, a00, A;
  double VI;                 /* Eq. 1, natural logarithm */
  double NMI;                /* Eq. 2; 1 when both partitions are a single community */
  double F;                  /* Eq. 3 (asymmetric: C is the reference) */
  double NVD;                /* Eq. 4 */
  double RI, ARI, JI;        /* Eqs. 5-7; ARI, JI are 1 when their denominators vanish */
  uint32_t device_flags;
  uint32_t reserved;
} cq_compare_result;

/* Optional export of the contingency table: DEVICE arrays of `capacity` entries,
 * one per non-zero cell (i, j, |c_i ∩ c'_j|), unspecified order. */
typedef struct {
  int32_t* ci;
  int32_t* cj;
  int64_t* count;
  int64_t capacity;
} cq_cell_table;

size_t cq_compare_workspace_size(int32_t n, int32_t num_labels_a, int32_t num_labels_b);

/*
 * Compare ground truth C (d_labels_a, DEVICE int32[n], values in [0, num_labels_a))
 * with detected C' (d_labels_b, DEVICE int32[n], values in [0, num_labels_b)).
 * n >= 2 (the pair count A = n(n-1)/2 must be positive).  Synchronous.
 */
cq_status cq_compare_partitions(cq_context* ctx, int32_t n, const int32_t* d_labels_a,
                                int32_t num_labels_a, const int32_t* d_labels_b, int32_t num_labels_b,
                                void* d_ws, size_t ws_bytes, cq_compare_result* h_out,
                                const cq_cell_table* cells);

/* Asynchronous form; result written to DEVICE memory d_out. */
cq_status cq_compare_partitions_async(cq_context* ctx, int32_t n, const int32_t* d_labels_a,
                                      int32_t num_labels_a, const int32_t* d_labels_b,
                                      int32_t num_labels_b, void* d_ws, size_t ws_bytes,
                                      cq_compare_result* d_out, const cq_cell_table* cells);

/* ---- serving (continuous batching) ----------------------------------------- */

/* A server keeps graphs resident (registered cq_graph handles), takes scoring and
 * comparison requests whose labels are in HOST memory, and runs them on the GPU as
 * soon as a slot and device memory are free, while other requests are still running:
 *   - each slot is one HIP stream, so launches of different slots overlap on the GPU;
 *   - a request is admitted when its footprint (labels + workspace + result) fits in
 *     the server's device arena (memory_budget bytes, allocated at creation);
 *   - small scoring requests (graph with <= small_nnz stored entries, num_labels <=
 *     16384) that are waiting together are grouped, up to max_batch, into one batched
 *     launch (the cq_batch kernels);
 *   - requests are otherwise served in arrival order.
 * Latency is measured from submit to the result being in host memory.  A request's
 * result is the same as that of the synchronous call on the same inputs. */
typedef struct cq_server cq_server;

typedef struct {
  int32_t num_slots;      /* launches in flight at once, >= 1 */
  int32_t max_batch;      /* most small scoring requests in one launch, >= 1 */
  int64_t memory_budget;  /* device bytes for request labels, workspaces and results */
  int64_t small_nnz;      /* graphs with at most this many stored entries are "small" */
} cq_server_config;

typedef struct {
  int64_t submitted, completed, failed, rejected;
  int64_t launches;          /* device launches (a grouped launch counts once) */
  int64_t grouped_requests;  /* requests that ran inside grouped launches */
  double p50_ms, p99_ms, mean_ms, max_ms;  /* submit -> result in host memory */
  double busy_s;             /* wall time with at least one launch in flight */
  int64_t peak_bytes;        /* most arena bytes admitted at once */
} cq_server_stats;

/* Create a server on ctx's device (it uses its own streams).  Allocates the arena,
 * pinned result buffers and starts one worker thread. */
cq_status cq_server_create(cq_context* ctx, const cq_server_config* cfg, cq_server** out);
/* Submit a scoring request.  h_labels: HOST int32[n] of graph g; it must stay valid
 * and unchanged until the request has been waited for (pinned memory transfers
 * fastest).  *ticket identifies the request.  CQ_E_BUSY: the request can never fit in
 * the arena. */
cq_status cq_server_submit_score(cq_server* srv, const cq_graph* g, const int32_t* h_labels, int32_t num_labels,
                                 uint64_t* ticket);
/* Submit a comparison request (HOST label arrays of length n, same lifetime rule). */
cq_status cq_server_submit_compare(cq_server* srv, int32_t n, const int32_t* h_labels_a, int32_t num_labels_a,
                                   const int32_t* h_labels_b, int32_t num_labels_b, uint64_t* ticket);
/* Wait up to timeout_ms (< 0: no limit) for a request, then release its ticket and
 * return its status and result (score_out or compare_out by kind; either may be NULL)
 * and its latency.  Returns CQ_E_BUSY if the request is not finished in time (the
 * ticket stays valid), CQ_E_INVALID_ARG for an unknown ticket or one another thread is
 * already waiting for. */
cq_status cq_server_wait(cq_server* srv, uint64_t ticket, double timeout_ms, cq_status* request_status,
                         cq_score_result* score_out, cq_compare_result* compare_out, double* latency_ms);
cq_status cq_server_get_stats(cq_server* srv, cq_server_stats* out);
cq_status cq_server_reset_stats(cq_server* srv);
/* Stop: waiting requests are cancelled (their status becomes CQ_E_CANCELLED), launches
 * in flight finish, threads blocked in cq_server_wait return (with the request's final
 * status), then everything is freed.  Tickets not yet waited for are lost.  No call on
 * srv may start once destroy has begun. */
void cq_server_destroy(cq_server* srv);

#ifdef __cplusplus
}
#endif
#endif /* CQ_H */
