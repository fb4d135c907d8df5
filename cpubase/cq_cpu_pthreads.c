/*
 * cq_cpu_pthreads.c -- multi-threaded CPU scoring of a partition (Q, Qds and the six
 * measures of Section II-B), organised the way the paper's shared-memory (Pthreads)
 * algorithm for the metrics without ground truth is: the community is the unit of
 * work, thread t owns the communities whose id is t modulo the thread count, and the
 * graph and the labels are shared by all threads (Section III-B, following the
 * community assignment of the distributed algorithm in Section III-A).
 *
 * BENCHMARK BASELINE ONLY.  It times the host's cores next to the GPU library; it is
 * not part of the library, which never calls it, and the oracle stays the reference
 * it is tested against.
 *
 * Steps:
 *   1. Members of every community: per-thread histograms of the labels over node
 *      ranges, prefix sums over (community, thread), then each thread places its
 *      nodes (a counting sort by label).
 *   2. Each thread walks the members of its communities: D_c (sum of degrees), the
 *      entries whose neighbour is in c (2|E_c^in|), and the counts |E_{c,j}| of every
 *      other neighbouring community j in a thread-private array of L counters (reset
 *      through the list of touched ids).  From them it forms the community's bracket of
 *      Eq. (8), its bracket of Eq. (9) with the split penalty sum_j |E_cj|/(2|E|) d_cj
 *      (d_cj = |E_cj| / (|c||j|)), and the six measures, accumulating them per thread
 *      with compensated sums.
 *   3. The per-thread sums are added in thread order.
 * Readings where the paper is silent are those of the library: d_c = 0 when |c| < 2,
 * conductance 0 when D_c = 0, label ids no node carries are not communities, means
 * are over the K non-empty communities.
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
  int64_t n, m, K, num_pairs, sum_ein, sum_eout;
  double Q, Qds, split_penalty;
  double mean_intra_edges, mean_intra_density, mean_contraction;
  double mean_inter_edges, mean_expansion, mean_conductance;
} cpu_score_result;

typedef struct {
  double s, c;
} csum;
static void cs_add(csum* a, double x) {
  const double t = a->s + x;
  a->c += fabs(a->s) >= fabs(x) ? (a->s - t) + x : (x - t) + a->s;
  a->s = t;
}
static double cs_val(const csum* a) { return a->s + a->c; }

enum { F_Q, F_QDS, F_PEN, F_IE, F_ID, F_CT, F_XE, F_EX, F_CO, F_COUNT };

typedef struct {
  /* shared inputs */
  int32_t n, L, T;
  const int32_t *rp, *col, *lab;
  int64_t m;
  int64_t* hist;   /* [L][T] label counts per thread's node range, then their places */
  int32_t* mem;    /* nodes grouped by label */
  int64_t* first;  /* first member of every label (L + 1) */
  /* per-thread state */
  int tid;
  int bad;
  int64_t K, pairs, sum_ein, sum_eout;
  csum f[F_COUNT];
} job;

static void range_of(int64_t total, int T, int t, int64_t* a, int64_t* b) {
  *a = total * t / T;
  *b = total * (t + 1) / T;
}

static void* count_labels(void* p) {
  job* j = (job*)p;
  int64_t a, b;
  range_of(j->n, j->T, j->tid, &a, &b);
  for (int64_t u = a; u < b; ++u) {
    const int32_t c = j->lab[u];
    if (c < 0 || c >= j->L) {
      j->bad = 1;
      return NULL;
    }
    ++j->hist[(int64_t)c * j->T + j->tid];
  }
  return NULL;
}

static void* place_nodes(void* p) {
  job* j = (job*)p;
  int64_t a, b;
  range_of(j->n, j->T, j->tid, &a, &b);
  for (int64_t u = a; u < b; ++u) {
    const int32_t c = j->lab[u];
    j->mem[j->hist[(int64_t)c * j->T + j->tid]++] = (int32_t)u;
  }
  return NULL;
}

static void* score_communities(void* p) {
  job* j = (job*)p;
  int64_t* cnt = calloc((size_t)j->L, sizeof(int64_t));
  int32_t* touched = malloc((size_t)j->L * sizeof(int32_t));
  if (!cnt || !touched) {
    j->bad = 2;
    free(cnt);
    free(touched);
    return NULL;
  }
  const double m = (double)j->m, twom = 2.0 * (double)j->m;
  for (int32_t c = j->tid; c < j->L; c += j->T) {  /* the paper's assignment: id mod threads */
    const int64_t b0 = j->first[c], b1 = j->first[c + 1];
    const int64_t nc = b1 - b0;
    if (nc == 0) continue;
    int64_t D = 0, I = 0;
    int32_t nt = 0;
    for (int64_t k = b0; k < b1; ++k) {
      const int32_t u = j->mem[k];
      const int32_t e0 = j->rp[u], e1 = j->rp[u + 1];
      D += e1 - e0;
      for (int32_t e = e0; e < e1; ++e) {
        const int32_t x = j->lab[j->col[e]];
        if (x == c) {
          ++I;
        } else {
          if (cnt[x] == 0) touched[nt++] = x;
          ++cnt[x];
        }
      }
    }
    const double ncd = (double)nc;
    const double ein = (double)(I / 2), eout = (double)(D - I);
    const double dc = nc >= 2 ? 2.0 * ein / (ncd * (ncd - 1.0)) : 0.0;
    /* split penalty of c: sum over neighbouring j of |E_cj|/(2|E|) * |E_cj|/(|c||j|) */
    csum pen = {0, 0};
    for (int32_t q = 0; q < nt; ++q) {
      const int32_t x = touched[q];
      const double ecj = (double)cnt[x];
      const double nj = (double)(j->first[x + 1] - j->first[x]);
      cs_add(&pen, (ecj / twom) * (ecj / (ncd * nj)));
      if (x > c) ++j->pairs;
      cnt[x] = 0;
    }
    const double pc = cs_val(&pen);
    const double dsum = (double)D;
    cs_add(&j->f[F_Q], ein / m - (dsum / twom) * (dsum / twom));
    cs_add(&j->f[F_QDS], (ein / m) * dc - (dsum * dc / twom) * (dsum * dc / twom) - pc);
    cs_add(&j->f[F_PEN], pc);
    cs_add(&j->f[F_IE], ein);
    cs_add(&j->f[F_ID], dc);
    cs_add(&j->f[F_CT], 2.0 * ein / ncd);
    cs_add(&j->f[F_XE], eout);
    cs_add(&j->f[F_EX], eout / ncd);
    cs_add(&j->f[F_CO], D > 0 ? eout / dsum : 0.0);
    ++j->K;
    j->sum_ein += I / 2;
    j->sum_eout += D - I;
  }
  free(cnt);
  free(touched);
  return NULL;
}

static int run_all(job* jobs, int T, void* (*fn)(void*)) {
  pthread_t* th = malloc((size_t)T * sizeof(pthread_t));
  if (!th) return -1;
  int started = 0, rc = 0;
  for (int t = 1; t < T; ++t) {
    if (pthread_create(&th[t], NULL, fn, &jobs[t]) != 0) {
      rc = -1;
      break;
    }
    started = t;
  }
  if (rc == 0) fn(&jobs[0]);
  for (int t = 1; t <= started; ++t) pthread_join(th[t], NULL);
  free(th);
  return rc;
}

/* Returns 0, or -1 (bad argument / no edges), -2 (label out of range), -11 (memory). */
int cpu_score(int32_t n, const int32_t* rp, const int32_t* col, const int32_t* lab, int32_t L, int32_t threads,
              cpu_score_result* out) {
  if (!out || n < 1 || L < 1 || threads < 1 || !rp || !col || !lab) return -1;
  memset(out, 0, sizeof(*out));
  const int64_t nnz = rp[n];
  if (nnz <= 0 || nnz % 2) return -1;
  const int T = threads > 256 ? 256 : threads;
  job* jobs = calloc((size_t)T, sizeof(job));
  int64_t* hist = calloc((size_t)L * T, sizeof(int64_t));
  int32_t* mem = malloc((size_t)n * sizeof(int32_t));
  int64_t* first = malloc(((size_t)L + 1) * sizeof(int64_t));
  int rc = 0;
  if (!jobs || !hist || !mem || !first) rc = -11;
  for (int t = 0; rc == 0 && t < T; ++t) {
    jobs[t] = (job){.n = n, .L = L, .T = T, .rp = rp, .col = col, .lab = lab, .m = nnz / 2,
                    .hist = hist, .mem = mem, .first = first, .tid = t};
  }
  if (rc == 0 && run_all(jobs, T, count_labels) != 0) rc = -11;
  for (int t = 0; rc == 0 && t < T; ++t)
    if (jobs[t].bad) rc = -2;
  if (rc == 0) {
    /* exclusive prefix over (label, thread): thread t's nodes of label c go after those
       of threads < t, so every label's members are contiguous */
    int64_t run = 0;
    for (int64_t c = 0; c < L; ++c) {
      first[c] = run;
      for (int t = 0; t < T; ++t) {
        const int64_t k = hist[c * T + t];
        hist[c * T + t] = run;
        run += k;
      }
    }
    first[L] = run;
    if (run_all(jobs, T, place_nodes) != 0 || run_all(jobs, T, score_communities) != 0) rc = -11;
    for (int t = 0; rc == 0 && t < T; ++t)
      if (jobs[t].bad) rc = -11;
  }
  if (rc == 0) {
    csum f[F_COUNT];
    memset(f, 0, sizeof(f));
    int64_t K = 0;
    for (int t = 0; t < T; ++t) {
      for (int k = 0; k < F_COUNT; ++k) cs_add(&f[k], cs_val(&jobs[t].f[k]));
      K += jobs[t].K;
      out->num_pairs += jobs[t].pairs;
      out->sum_ein += jobs[t].sum_ein;
      out->sum_eout += jobs[t].sum_eout;
    }
    out->n = n;
    out->m = nnz / 2;
    out->K = K;
    out->Q = cs_val(&f[F_Q]);
    out->Qds = cs_val(&f[F_QDS]);
    out->split_penalty = cs_val(&f[F_PEN]);
    out->mean_intra_edges = cs_val(&f[F_IE]) / (double)K;
    out->mean_intra_density = cs_val(&f[F_ID]) / (double)K;
    out->mean_contraction = cs_val(&f[F_CT]) / (double)K;
    out->mean_inter_edges = cs_val(&f[F_XE]) / (double)K;
    out->mean_expansion = cs_val(&f[F_EX]) / (double)K;
    out->mean_conductance = cs_val(&f[F_CO]) / (double)K;
  }
  free(jobs);
  free(hist);
  free(mem);
  free(first);
  return rc;
}
