/*
 * cq_oracle.c -- plain, slow, obviously-correct CPU oracle for community-quality
 * metrics (Chen, Liu, Szymanski, "Parallel Toolkit for Measuring the Quality of
 * Network Community Structure").
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the independent reference against which
 * the GPU library is checked.  It shares no code, header, table or helper with the
 * GPU path, and the GPU path never calls it.  Only the test suite, the smoke check
 * and the benchmark's CPU-baseline leg may load it.
 *
 * Every quantity is computed the way the paper defines it:
 *   score   -- Section II-B: modularity Q (Eq. 8), modularity density Qds (Eq. 9,
 *              with the internal density d_c and the pair density d_{ci,cj}), and the
 *              six per-community measures of Section II-B3 (intra-edges, intra-density,
 *              contraction, inter-edges, expansion, conductance).
 *   compare -- Section II-A: VI (Eq. 1), NMI (Eq. 2), F-measure (Eq. 3), NVD (Eq. 4),
 *              and the pair-counting metrics RI, ARI, JI (Eqs. 5-7) from the pair
 *              counts a11, a10, a01, a00 defined in Section II-A3.
 *
 * Readings where the paper is silent (each one is also listed in the design notes):
 *   - d_c = 0 for a community with fewer than two nodes (0/0 in Eq. 9).
 *   - conductance = 0 for a community whose degree sum is 0.
 *   - |E_{ci,cj}| is the number of undirected edges with one end in ci and the other
 *     in cj; the inner sum of Eq. 9 runs over ordered pairs (ci, cj), cj != ci.
 *   - label ids that no node carries are not communities: they are excluded from
 *     every sum and from the community count K.
 *   - the six measures are reported per community and as unweighted means over the
 *     K non-empty communities.
 *   - NMI = 1 when both entropies are zero (both partitions are one community);
 *     ARI = 1 and JI = 1 when their denominators are zero (identical partitions).
 *   - pair counts are unordered node pairs, A = |V|(|V|-1)/2 (Section II-A3).
 *   - logarithms are natural (the paper does not fix a base; NMI does not depend
 *     on it, VI is reported in nats).
 *
 * The pair counts a11..a00 are obtained from the contingency table
 * (a11 = sum over cells of C(n_ij, 2), a10 = sum_i C(|c_i|, 2) - a11, ...).  This is
 * the counting identity behind the definitions of Section II-A3; the tests pin it
 * against explicit enumeration of all node pairs on small inputs.
 *
 * All floating-point sums use Neumaier (compensated) summation in binary64 over
 * terms evaluated in binary64, accumulated in ascending label order.
 *
 * Weighted score (orc_score_w).  The paper defines Eqs. 8-9 for unweighted graphs and
 * notes (for weighted ones) that the two densities keep unweighted edge counts, so
 * that they never exceed 1.  Reading used here, for a symmetric positive weight w(e)
 * per CSR entry:
 *   - every edge count of Eqs. 8-9 that is not inside a density becomes a weight sum:
 *     |E| -> W (sum of the weights of the undirected edges), |E_c^in| -> w_in(c),
 *     |E_c^out| -> w_out(c), 2|E_c^in| + |E_c^out| -> s(c) (the strength sum of c),
 *     |E_{ci,cj}| in front of d_{ci,cj} -> w(ci,cj);
 *   - d_c and d_{ci,cj} use the unweighted counts, as in the unweighted case;
 *   - the six measures: intra-edges w_in(c), intra-density d_c, contraction
 *     2 w_in(c)/|c|, inter-edges w_out(c), expansion w_out(c)/|c|, conductance
 *     w_out(c)/s(c) (0 when s(c) = 0).
 * With every weight equal to 1 this is exactly the unweighted score.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>

#define ORC_OK 0
#define ORC_E_ARG (-1)
#define ORC_E_LABEL (-2)
#define ORC_E_GRAPH (-3)
#define ORC_E_NOEDGES (-6)
#define ORC_E_CAPACITY (-10)
#define ORC_E_NOMEM (-11)

typedef struct {
  int64_t n;               /* |V| */
  int64_t m;               /* |E|, undirected edges */
  int64_t K;               /* non-empty communities */
  int64_t num_pairs;       /* unordered community pairs with |E_{ci,cj}| > 0 */
  int64_t sum_ein;         /* sum over c of |E_c^in| */
  int64_t sum_eout;        /* sum over c of |E_c^out| */
  double Q;                /* Eq. 8 */
  double Qds;              /* Eq. 9 */
  double split_penalty;    /* sum_i sum_{j!=i} |E_ij|/(2|E|) * d_ij (the subtracted part of Eq. 9) */
  double mean_intra_edges;
  double mean_intra_density;
  double mean_contraction;
  double mean_inter_edges;
  double mean_expansion;
  double mean_conductance;
} orc_score_result;

typedef struct {
  int64_t n;               /* |V| */
  int64_t Ka, Kb;          /* non-empty communities in C and C' */
  int64_t nnz;             /* cells with |c ∩ c'| > 0 */
  int64_t a11, a10, a01, a00, A;
  double VI, NMI, F, NVD, RI, ARI, JI;
} orc_compare_result;

/* ---- compensated summation ------------------------------------------------ */
typedef struct { double s, c; } nsum;
static void ns_add(nsum* a, double x) {
  double t = a->s + x;
  if (fabs(a->s) >= fabs(x)) a->c += (a->s - t) + x;
  else a->c += (x - t) + a->s;
  a->s = t;
}
static double ns_get(const nsum* a) { return a->s + a->c; }

static int cmp_u64(const void* x, const void* y) {
  uint64_t a = *(const uint64_t*)x, b = *(const uint64_t*)y;
  return (a > b) - (a < b);
}

/* ---- score (Section II-B) ------------------------------------------------- */
/*
 * Inputs: symmetric CSR of a simple undirected graph (row_ptr[n+1], col_idx[row_ptr[n]]),
 * labels[n] in [0, L).  Optional outputs (NULL to skip), per label id, length L:
 * size, degsum (sum of degrees = 2|E_in| + |E_out|), ein, eout, intra_density,
 * contraction, expansion, conductance, q_term (bracket of Eq. 8), qds_term (bracket
 * of Eq. 9).  Optional pair table (pair_cap > 0): unordered pairs (ci < cj) with
 * their edge counts, ascending by (ci, cj).
 */
int orc_score(int32_t n, const int32_t* row_ptr, const int32_t* col_idx,
              const int32_t* labels, int32_t L, orc_score_result* out,
              int64_t* size, int64_t* degsum, int64_t* ein, int64_t* eout,
              double* intra_density, double* contraction, double* expansion,
              double* conductance, double* q_term, double* qds_term,
              int32_t* pair_i, int32_t* pair_j, int64_t* pair_cnt, int64_t pair_cap) {
  if (!out || n < 1 || L < 1 || !row_ptr || !col_idx || !labels) return ORC_E_ARG;
  memset(out, 0, sizeof(*out));
  int64_t nnz = row_ptr[n];
  if (row_ptr[0] != 0 || nnz < 0) return ORC_E_GRAPH;
  for (int32_t u = 0; u < n; ++u)
    if (row_ptr[u + 1] < row_ptr[u]) return ORC_E_GRAPH;
  for (int64_t e = 0; e < nnz; ++e)
    if (col_idx[e] < 0 || col_idx[e] >= n) return ORC_E_GRAPH;
  for (int32_t u = 0; u < n; ++u)
    if (labels[u] < 0 || labels[u] >= L) return ORC_E_LABEL;
  if (nnz % 2 != 0) return ORC_E_GRAPH;
  int64_t m = nnz / 2;            /* each undirected edge appears twice in the CSR */
  if (m == 0) return ORC_E_NOEDGES;

  int64_t* nc = calloc((size_t)L, sizeof(int64_t));    /* |c| */
  int64_t* in2 = calloc((size_t)L, sizeof(int64_t));   /* 2|E_c^in|: internal CSR entries */
  int64_t* outc = calloc((size_t)L, sizeof(int64_t));  /* |E_c^out|: boundary CSR entries */
  double* dens = calloc((size_t)L, sizeof(double));
  nsum* pen = calloc((size_t)L, sizeof(nsum));         /* inner sum of Eq. 9 for each c_i */
  if (!nc || !in2 || !outc || !dens || !pen) {
    free(nc); free(in2); free(outc); free(dens); free(pen); return ORC_E_NOMEM;
  }

  /* community sizes */
  for (int32_t u = 0; u < n; ++u) nc[labels[u]] += 1;

  /* walk every edge end: an edge u-v with both ends in c is inside c (counted once from
   * each end, so in2 holds 2|E_c^in|); otherwise it is on the boundary of c. */
  int64_t nkeys = 0;
  for (int32_t u = 0; u < n; ++u) {
    int32_t cu = labels[u];
    for (int64_t e = row_ptr[u]; e < row_ptr[u + 1]; ++e) {
      int32_t cv = labels[col_idx[e]];
      if (cv == cu) in2[cu] += 1;
      else { outc[cu] += 1; if (cu < cv) ++nkeys; }
    }
  }
  /* |E_{ci,cj}|: list every undirected boundary edge once (from the end in the lower
   * community id), sort, count runs. */
  uint64_t* keys = malloc((size_t)(nkeys > 0 ? nkeys : 1) * sizeof(uint64_t));
  if (!keys) { free(nc); free(in2); free(outc); free(dens); free(pen); return ORC_E_NOMEM; }
  int64_t kk = 0;
  for (int32_t u = 0; u < n; ++u) {
    int32_t cu = labels[u];
    for (int64_t e = row_ptr[u]; e < row_ptr[u + 1]; ++e) {
      int32_t cv = labels[col_idx[e]];
      if (cu < cv) keys[kk++] = ((uint64_t)(uint32_t)cu << 32) | (uint32_t)cv;
    }
  }
  qsort(keys, (size_t)nkeys, sizeof(uint64_t), cmp_u64);

  /* internal densities d_c (Eq. 9) */
  for (int32_t c = 0; c < L; ++c) {
    int64_t e_in = in2[c] / 2;
    dens[c] = nc[c] >= 2 ? (2.0 * (double)e_in) / ((double)nc[c] * (double)(nc[c] - 1)) : 0.0;
  }

  /* split penalty: for each unordered pair {ci, cj} the term |E_ij|/(2|E|) * d_ij appears
   * in the bracket of ci and in the bracket of cj (ordered pairs). */
  int64_t npairs = 0;
  int rc = ORC_OK;
  for (int64_t a = 0; a < nkeys;) {
    int64_t b = a;
    while (b < nkeys && keys[b] == keys[a]) ++b;
    int32_t ci = (int32_t)(keys[a] >> 32), cj = (int32_t)(keys[a] & 0xffffffffu);
    int64_t eij = b - a;
    double dij = (double)eij / ((double)nc[ci] * (double)nc[cj]);
    double term = (double)eij / (2.0 * (double)m) * dij;
    ns_add(&pen[ci], term);
    ns_add(&pen[cj], term);
    if (pair_cap > 0) {
      if (npairs < pair_cap) { pair_i[npairs] = ci; pair_j[npairs] = cj; pair_cnt[npairs] = eij; }
      else rc = ORC_E_CAPACITY;
    }
    ++npairs;
    a = b;
  }
  free(keys);

  nsum q = {0, 0}, qds = {0, 0}, ptot = {0, 0};
  nsum s_dens = {0, 0}, s_contr = {0, 0}, s_exp = {0, 0}, s_cond = {0, 0};
  int64_t K = 0, sum_ein = 0, sum_eout = 0;
  for (int32_t c = 0; c < L; ++c) {
    int64_t e_in = in2[c] / 2, e_out = outc[c];
    double qt = 0.0, qdt = 0.0, contr = 0.0, expa = 0.0, cond = 0.0;
    if (nc[c] > 0) {
      ++K;
      sum_ein += e_in;
      sum_eout += e_out;
      double tot = (double)(2 * e_in + e_out) / (2.0 * (double)m);
      /* Eq. 8 bracket */
      qt = (double)e_in / (double)m - tot * tot;
      /* Eq. 9 bracket */
      double tdc = tot * dens[c];
      qdt = (double)e_in / (double)m * dens[c] - tdc * tdc - ns_get(&pen[c]);
      contr = 2.0 * (double)e_in / (double)nc[c];
      expa = (double)e_out / (double)nc[c];
      cond = (2 * e_in + e_out) > 0 ? (double)e_out / (double)(2 * e_in + e_out) : 0.0;
      ns_add(&q, qt);
      ns_add(&qds, qdt);
      ns_add(&ptot, ns_get(&pen[c]));
      ns_add(&s_dens, dens[c]);
      ns_add(&s_contr, contr);
      ns_add(&s_exp, expa);
      ns_add(&s_cond, cond);
    }
    if (size) size[c] = nc[c];
    if (degsum) degsum[c] = 2 * e_in + e_out;
    if (ein) ein[c] = e_in;
    if (eout) eout[c] = e_out;
    if (intra_density) intra_density[c] = dens[c];
    if (contraction) contraction[c] = contr;
    if (expansion) expansion[c] = expa;
    if (conductance) conductance[c] = cond;
    if (q_term) q_term[c] = qt;
    if (qds_term) qds_term[c] = qdt;
  }
  out->n = n;
  out->m = m;
  out->K = K;
  out->num_pairs = npairs;
  out->sum_ein = sum_ein;
  out->sum_eout = sum_eout;
  out->Q = ns_get(&q);
  out->Qds = ns_get(&qds);
  out->split_penalty = ns_get(&ptot);
  out->mean_intra_edges = (double)sum_ein / (double)K;
  out->mean_intra_density = ns_get(&s_dens) / (double)K;
  out->mean_contraction = ns_get(&s_contr) / (double)K;
  out->mean_inter_edges = (double)sum_eout / (double)K;
  out->mean_expansion = ns_get(&s_exp) / (double)K;
  out->mean_conductance = ns_get(&s_cond) / (double)K;
  free(nc); free(in2); free(outc); free(dens); free(pen);
  return rc;
}

/* ---- weighted score (Section II-B with edge weights, see the reading above) -- */
typedef struct {
  int64_t n, m, K, num_pairs, sum_ein, sum_eout;   /* unweighted counts, as in orc_score */
  double W;                /* sum of the weights of the undirected edges */
  double sum_w_in;         /* sum over c of w_in(c) */
  double sum_w_out;        /* sum over c of w_out(c) */
  double Q, Qds, split_penalty;
  double mean_intra_edges, mean_intra_density, mean_contraction;
  double mean_inter_edges, mean_expansion, mean_conductance;
} orc_score_w_result;

/*
 * Same graph and label contract as orc_score plus w[row_ptr[n]]: one weight per CSR
 * entry, finite and > 0, equal for the two entries of an undirected edge.  Optional
 * per-label outputs (length L): strength s(c), w_in(c), w_out(c), intra_density (d_c,
 * unweighted), contraction, expansion, conductance, q_term, qds_term (weighted).
 * Optional pair table: unordered pairs (ci < cj) with |E_{ci,cj}| and w(ci,cj),
 * ascending by (ci, cj).
 */
typedef struct { uint64_t key; double w; } orc_wkey;
static int cmp_wkey(const void* x, const void* y) {
  uint64_t a = ((const orc_wkey*)x)->key, b = ((const orc_wkey*)y)->key;
  return (a > b) - (a < b);
}

int orc_score_w(int32_t n, const int32_t* row_ptr, const int32_t* col_idx, const float* w,
                const int32_t* labels, int32_t L, orc_score_w_result* out,
                double* strength, double* w_in, double* w_out, double* intra_density,
                double* contraction, double* expansion, double* conductance, double* q_term,
                double* qds_term, int32_t* pair_i, int32_t* pair_j, int64_t* pair_cnt,
                double* pair_w, int64_t pair_cap) {
  if (!out || n < 1 || L < 1 || !row_ptr || !col_idx || !labels || !w) return ORC_E_ARG;
  memset(out, 0, sizeof(*out));
  int64_t nnz = row_ptr[n];
  if (row_ptr[0] != 0 || nnz < 0) return ORC_E_GRAPH;
  for (int32_t u = 0; u < n; ++u)
    if (row_ptr[u + 1] < row_ptr[u]) return ORC_E_GRAPH;
  for (int64_t e = 0; e < nnz; ++e) {
    if (col_idx[e] < 0 || col_idx[e] >= n) return ORC_E_GRAPH;
    if (!(w[e] > 0.0f) || !isfinite(w[e])) return ORC_E_GRAPH;
  }
  for (int32_t u = 0; u < n; ++u)
    if (labels[u] < 0 || labels[u] >= L) return ORC_E_LABEL;
  if (nnz % 2 != 0) return ORC_E_GRAPH;
  int64_t m = nnz / 2;
  if (m == 0) return ORC_E_NOEDGES;

  int64_t* nc = calloc((size_t)L, sizeof(int64_t));   /* |c| */
  int64_t* in2 = calloc((size_t)L, sizeof(int64_t));  /* 2|E_c^in| (unweighted) */
  int64_t* outc = calloc((size_t)L, sizeof(int64_t)); /* |E_c^out| (unweighted) */
  nsum* s_c = calloc((size_t)L, sizeof(nsum));        /* s(c) */
  nsum* win2 = calloc((size_t)L, sizeof(nsum));       /* 2 w_in(c) */
  nsum* wout = calloc((size_t)L, sizeof(nsum));       /* w_out(c) */
  double* dens = calloc((size_t)L, sizeof(double));
  nsum* pen = calloc((size_t)L, sizeof(nsum));
  if (!nc || !in2 || !outc || !s_c || !win2 || !wout || !dens || !pen) {
    free(nc); free(in2); free(outc); free(s_c); free(win2); free(wout); free(dens); free(pen);
    return ORC_E_NOMEM;
  }
  for (int32_t u = 0; u < n; ++u) nc[labels[u]] += 1;
  nsum Wsum = {0, 0};
  int64_t nkeys = 0;
  for (int32_t u = 0; u < n; ++u) {
    int32_t cu = labels[u];
    for (int64_t e = row_ptr[u]; e < row_ptr[u + 1]; ++e) {
      int32_t cv = labels[col_idx[e]];
      double we = (double)w[e];
      ns_add(&Wsum, we);
      ns_add(&s_c[cu], we);
      if (cv == cu) { in2[cu] += 1; ns_add(&win2[cu], we); }
      else { outc[cu] += 1; ns_add(&wout[cu], we); if (cu < cv) ++nkeys; }
    }
  }
  double W = ns_get(&Wsum) / 2.0;  /* every undirected edge is stored twice */
  orc_wkey* keys = malloc((size_t)(nkeys > 0 ? nkeys : 1) * sizeof(orc_wkey));
  if (!keys) {
    free(nc); free(in2); free(outc); free(s_c); free(win2); free(wout); free(dens); free(pen);
    return ORC_E_NOMEM;
  }
  int64_t kk = 0;
  for (int32_t u = 0; u < n; ++u) {
    int32_t cu = labels[u];
    for (int64_t e = row_ptr[u]; e < row_ptr[u + 1]; ++e) {
      int32_t cv = labels[col_idx[e]];
      if (cu < cv) {
        keys[kk].key = ((uint64_t)(uint32_t)cu << 32) | (uint32_t)cv;
        keys[kk].w = (double)w[e];
        ++kk;
      }
    }
  }
  qsort(keys, (size_t)nkeys, sizeof(orc_wkey), cmp_wkey);
  for (int32_t c = 0; c < L; ++c) {
    int64_t e_in = in2[c] / 2;
    dens[c] = nc[c] >= 2 ? (2.0 * (double)e_in) / ((double)nc[c] * (double)(nc[c] - 1)) : 0.0;  /* unweighted count */
  }
  int64_t npairs = 0;
  int rc = ORC_OK;
  for (int64_t a = 0; a < nkeys;) {
    int64_t b = a;
    nsum wij = {0, 0};
    while (b < nkeys && keys[b].key == keys[a].key) { ns_add(&wij, keys[b].w); ++b; }
    int32_t ci = (int32_t)(keys[a].key >> 32), cj = (int32_t)(keys[a].key & 0xffffffffu);
    int64_t eij = b - a;
    double dij = (double)eij / ((double)nc[ci] * (double)nc[cj]);   /* unweighted density */
    double term = ns_get(&wij) / (2.0 * W) * dij;                  /* weighted fraction */
    ns_add(&pen[ci], term);
    ns_add(&pen[cj], term);
    if (pair_cap > 0) {
      if (npairs < pair_cap) {
        pair_i[npairs] = ci; pair_j[npairs] = cj; pair_cnt[npairs] = eij;
        if (pair_w) pair_w[npairs] = ns_get(&wij);
      } else {
        rc = ORC_E_CAPACITY;
      }
    }
    ++npairs;
    a = b;
  }
  free(keys);

  nsum q = {0, 0}, qds = {0, 0}, ptot = {0, 0}, swin = {0, 0}, swout = {0, 0};
  nsum s_dens = {0, 0}, s_contr = {0, 0}, s_exp = {0, 0}, s_cond = {0, 0};
  int64_t K = 0, sum_ein = 0, sum_eout = 0;
  for (int32_t c = 0; c < L; ++c) {
    double wi = ns_get(&win2[c]) / 2.0, wo = ns_get(&wout[c]), sc = ns_get(&s_c[c]);
    double qt = 0.0, qdt = 0.0, contr = 0.0, expa = 0.0, cond = 0.0;
    if (nc[c] > 0) {
      ++K;
      sum_ein += in2[c] / 2;
      sum_eout += outc[c];
      double tot = sc / (2.0 * W);
      qt = wi / W - tot * tot;
      double tdc = tot * dens[c];
      qdt = wi / W * dens[c] - tdc * tdc - ns_get(&pen[c]);
      contr = 2.0 * wi / (double)nc[c];
      expa = wo / (double)nc[c];
      cond = sc > 0.0 ? wo / sc : 0.0;
      ns_add(&q, qt);
      ns_add(&qds, qdt);
      ns_add(&ptot, ns_get(&pen[c]));
      ns_add(&swin, wi);
      ns_add(&swout, wo);
      ns_add(&s_dens, dens[c]);
      ns_add(&s_contr, contr);
      ns_add(&s_exp, expa);
      ns_add(&s_cond, cond);
    }
    if (strength) strength[c] = sc;
    if (w_in) w_in[c] = wi;
    if (w_out) w_out[c] = wo;
    if (intra_density) intra_density[c] = dens[c];
    if (contraction) contraction[c] = contr;
    if (expansion) expansion[c] = expa;
    if (conductance) conductance[c] = cond;
    if (q_term) q_term[c] = qt;
    if (qds_term) qds_term[c] = qdt;
  }
  out->n = n;
  out->m = m;
  out->K = K;
  out->num_pairs = npairs;
  out->sum_ein = sum_ein;
  out->sum_eout = sum_eout;
  out->W = W;
  out->sum_w_in = ns_get(&swin);
  out->sum_w_out = ns_get(&swout);
  out->Q = ns_get(&q);
  out->Qds = ns_get(&qds);
  out->split_penalty = ns_get(&ptot);
  out->mean_intra_edges = ns_get(&swin) / (double)K;
  out->mean_intra_density = ns_get(&s_dens) / (double)K;
  out->mean_contraction = ns_get(&s_contr) / (double)K;
  out->mean_inter_edges = ns_get(&swout) / (double)K;
  out->mean_expansion = ns_get(&s_exp) / (double)K;
  out->mean_conductance = ns_get(&s_cond) / (double)K;
  free(nc); free(in2); free(outc); free(s_c); free(win2); free(wout); free(dens); free(pen);
  return rc;
}

/* ---- compare (Section II-A) ----------------------------------------------- */
static int64_t choose2(int64_t x) { return x * (x - 1) / 2; }

/*
 * Ground truth C = labels a (ids in [0, La)), detected C' = labels b (ids in [0, Lb)),
 * over the same N >= 2 nodes.  Optional cell output (cap > 0): the non-zero cells
 * |c_i ∩ c'_j| ascending by (i, j).
 */
int orc_compare(int32_t N, const int32_t* la, int32_t La, const int32_t* lb, int32_t Lb,
                orc_compare_result* out, int32_t* cell_i, int32_t* cell_j, int64_t* cell_n,
                int64_t cap) {
  if (!out || !la || !lb || N < 2 || La < 1 || Lb < 1) return ORC_E_ARG;
  memset(out, 0, sizeof(*out));
  for (int32_t u = 0; u < N; ++u)
    if (la[u] < 0 || la[u] >= La || lb[u] < 0 || lb[u] >= Lb) return ORC_E_LABEL;

  int64_t* a = calloc((size_t)La, sizeof(int64_t));    /* |c| for c in C */
  int64_t* b = calloc((size_t)Lb, sizeof(int64_t));    /* |c'| for c' in C' */
  int64_t* rowmax = calloc((size_t)La, sizeof(int64_t));
  double* rowf = calloc((size_t)La, sizeof(double));
  int64_t* colmax = calloc((size_t)Lb, sizeof(int64_t));
  uint64_t* keys = malloc((size_t)N * sizeof(uint64_t));
  if (!a || !b || !rowmax || !rowf || !colmax || !keys) {
    free(a); free(b); free(rowmax); free(rowf); free(colmax); free(keys); return ORC_E_NOMEM;
  }
  for (int32_t u = 0; u < N; ++u) {
    a[la[u]] += 1;
    b[lb[u]] += 1;
    keys[u] = ((uint64_t)(uint32_t)la[u] << 32) | (uint32_t)lb[u];
  }
  qsort(keys, (size_t)N, sizeof(uint64_t), cmp_u64);

  const double Nd = (double)N;
  nsum mi = {0, 0}, vi = {0, 0};
  int64_t a11 = 0, nnz = 0;
  int rc = ORC_OK;
  for (int64_t s = 0; s < N;) {
    int64_t t = s;
    while (t < N && keys[t] == keys[s]) ++t;
    int32_t i = (int32_t)(keys[s] >> 32), j = (int32_t)(keys[s] & 0xffffffffu);
    int64_t nij = t - s;                        /* |c_i ∩ c'_j| */
    /* Eq. 2 numerator term (without the -2) and Eq. 1 term (without the -1/|V|) */
    ns_add(&mi, (double)nij / Nd * log((double)nij * Nd / ((double)a[i] * (double)b[j])));
    ns_add(&vi, (double)nij * log((double)nij * (double)nij / ((double)a[i] * (double)b[j])));
    /* Eq. 3: max over c' of 2|c ∩ c'|/(|c| + |c'|); Eq. 4: maxima of |c ∩ c'| */
    double f = 2.0 * (double)nij / (double)(a[i] + b[j]);
    if (f > rowf[i]) rowf[i] = f;
    if (nij > rowmax[i]) rowmax[i] = nij;
    if (nij > colmax[j]) colmax[j] = nij;
    a11 += choose2(nij);
    if (cap > 0) {
      if (nnz < cap) { cell_i[nnz] = i; cell_j[nnz] = j; cell_n[nnz] = nij; }
      else rc = ORC_E_CAPACITY;
    }
    ++nnz;
    s = t;
  }
  free(keys);

  nsum ha = {0, 0}, hb = {0, 0}, fs = {0, 0};
  int64_t Ka = 0, Kb = 0, X = 0, Y = 0, sum_rowmax = 0, sum_colmax = 0;
  for (int32_t i = 0; i < La; ++i) {
    if (a[i] == 0) continue;
    ++Ka;
    ns_add(&ha, (double)a[i] / Nd * log((double)a[i] / Nd));
    ns_add(&fs, (double)a[i] * rowf[i]);
    sum_rowmax += rowmax[i];
    X += choose2(a[i]);
  }
  for (int32_t j = 0; j < Lb; ++j) {
    if (b[j] == 0) continue;
    ++Kb;
    ns_add(&hb, (double)b[j] / Nd * log((double)b[j] / Nd));
    sum_colmax += colmax[j];
    Y += choose2(b[j]);
  }
  /* Section II-A3 pair counts */
  int64_t A = choose2((int64_t)N);
  int64_t a10 = X - a11, a01 = Y - a11, a00 = A - a11 - a10 - a01;

  out->n = N;
  out->Ka = Ka;
  out->Kb = Kb;
  out->nnz = nnz;
  out->a11 = a11; out->a10 = a10; out->a01 = a01; out->a00 = a00; out->A = A;
  out->VI = -ns_get(&vi) / Nd;                                   /* Eq. 1 */
  double den = ns_get(&ha) + ns_get(&hb);
  out->NMI = den != 0.0 ? (-2.0 * ns_get(&mi)) / den : 1.0;     /* Eq. 2 */
  out->F = ns_get(&fs) / Nd;                                     /* Eq. 3 */
  out->NVD = 1.0 - (double)(sum_rowmax + sum_colmax) / (2.0 * Nd);   /* Eq. 4 */
  out->RI = (double)(a11 + a00) / (double)A;                     /* Eq. 5 */
  {                                                              /* Eq. 6 */
    double M = (double)(a11 + a10) * (double)(a11 + a01) / (double)A;
    double dd = 0.5 * ((double)(a11 + a10) + (double)(a11 + a01)) - M;
    out->ARI = dd != 0.0 ? ((double)a11 - M) / dd : 1.0;
  }
  {                                                              /* Eq. 7 */
    int64_t dj = a11 + a10 + a01;
    out->JI = dj != 0 ? (double)a11 / (double)dj : 1.0;
  }
  free(a); free(b); free(rowmax); free(rowf); free(colmax);
  return rc;
}
