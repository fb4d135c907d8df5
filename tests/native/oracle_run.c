/* Runs the CPU oracle once on an input file and prints every result exactly (host test
 * infrastructure, see host_input.h).  Built with the address and undefined-behaviour
 * sanitizers by tests/test_host_sanitized.py, which compares the printout with the
 * normally built oracle's results.  Every output array is allocated at exactly the
 * length the oracle's contract gives it (num_labels per community array, the pair and
 * cell tables at their stated capacity), so a write past it is caught. */
#include "cq_oracle.c"
#include "host_input.h"

static int64_t pair_capacity(int64_t nnz, int32_t L) {
  const int64_t m = nnz / 2, all = (int64_t)L * (L - 1) / 2;
  return m < all ? m : all;
}

static void run_score(const host_input* in) {
  const int32_t L = in->L;
  int64_t* ia[4];
  double* da[6];
  for (int k = 0; k < 4; ++k) ia[k] = malloc((size_t)L * sizeof(int64_t));
  for (int k = 0; k < 6; ++k) da[k] = malloc((size_t)L * sizeof(double));
  const int64_t cap = pair_capacity(in->nnz, L);
  int32_t* pi = cap ? malloc((size_t)cap * 4) : NULL;
  int32_t* pj = cap ? malloc((size_t)cap * 4) : NULL;
  int64_t* pc = cap ? malloc((size_t)cap * 8) : NULL;
  orc_score_result r;
  const int rc = orc_score(in->n, in->rp, in->ci, in->lab, L, &r, ia[0], ia[1], ia[2], ia[3], da[0], da[1], da[2],
                           da[3], da[4], da[5], pi, pj, pc, cap);
  put_i("rc", rc);
  if (rc == ORC_OK) {
    put_i("n", r.n), put_i("m", r.m), put_i("K", r.K), put_i("num_pairs", r.num_pairs);
    put_i("sum_ein", r.sum_ein), put_i("sum_eout", r.sum_eout);
    put_d("Q", r.Q), put_d("Qds", r.Qds), put_d("split_penalty", r.split_penalty);
    put_d("mean_intra_edges", r.mean_intra_edges), put_d("mean_intra_density", r.mean_intra_density);
    put_d("mean_contraction", r.mean_contraction), put_d("mean_inter_edges", r.mean_inter_edges);
    put_d("mean_expansion", r.mean_expansion), put_d("mean_conductance", r.mean_conductance);
    const char* in_names[4] = {"size", "degsum", "ein", "eout"};
    const char* d_names[6] = {"intra_density", "contraction", "expansion", "conductance", "q_term", "qds_term"};
    for (int k = 0; k < 4; ++k) put_h(in_names[k], ia[k], (size_t)L * 8);
    for (int k = 0; k < 6; ++k) put_h(d_names[k], da[k], (size_t)L * 8);
    put_h("pair_i", pi, (size_t)r.num_pairs * 4), put_h("pair_j", pj, (size_t)r.num_pairs * 4);
    put_h("pair_cnt", pc, (size_t)r.num_pairs * 8);
  }
  for (int k = 0; k < 4; ++k) free(ia[k]);
  for (int k = 0; k < 6; ++k) free(da[k]);
  free(pi), free(pj), free(pc);
}

static void run_score_w(const host_input* in) {
  const int32_t L = in->L;
  double* da[9];
  for (int k = 0; k < 9; ++k) da[k] = malloc((size_t)L * sizeof(double));
  const int64_t cap = pair_capacity(in->nnz, L);
  int32_t* pi = cap ? malloc((size_t)cap * 4) : NULL;
  int32_t* pj = cap ? malloc((size_t)cap * 4) : NULL;
  int64_t* pc = cap ? malloc((size_t)cap * 8) : NULL;
  double* pw = cap ? malloc((size_t)cap * 8) : NULL;
  orc_score_w_result r;
  const int rc = orc_score_w(in->n, in->rp, in->ci, in->w, in->lab, L, &r, da[0], da[1], da[2], da[3], da[4], da[5],
                             da[6], da[7], da[8], pi, pj, pc, pw, cap);
  put_i("rc", rc);
  if (rc == ORC_OK) {
    put_i("n", r.n), put_i("m", r.m), put_i("K", r.K), put_i("num_pairs", r.num_pairs);
    put_i("sum_ein", r.sum_ein), put_i("sum_eout", r.sum_eout);
    put_d("W", r.W), put_d("sum_w_in", r.sum_w_in), put_d("sum_w_out", r.sum_w_out);
    put_d("Q", r.Q), put_d("Qds", r.Qds), put_d("split_penalty", r.split_penalty);
    put_d("mean_intra_edges", r.mean_intra_edges), put_d("mean_intra_density", r.mean_intra_density);
    put_d("mean_contraction", r.mean_contraction), put_d("mean_inter_edges", r.mean_inter_edges);
    put_d("mean_expansion", r.mean_expansion), put_d("mean_conductance", r.mean_conductance);
    const char* d_names[9] = {"strength", "w_in", "w_out", "intra_density", "contraction",
                              "expansion", "conductance", "q_term", "qds_term"};
    for (int k = 0; k < 9; ++k) put_h(d_names[k], da[k], (size_t)L * 8);
    put_h("pair_i", pi, (size_t)r.num_pairs * 4), put_h("pair_j", pj, (size_t)r.num_pairs * 4);
    put_h("pair_cnt", pc, (size_t)r.num_pairs * 8), put_h("pair_w", pw, (size_t)r.num_pairs * 8);
  }
  for (int k = 0; k < 9; ++k) free(da[k]);
  free(pi), free(pj), free(pc), free(pw);
}

static void run_compare(const host_input* in) {
  const int64_t cap = in->n;
  int32_t* ci = malloc((size_t)cap * 4);
  int32_t* cj = malloc((size_t)cap * 4);
  int64_t* cn = malloc((size_t)cap * 8);
  orc_compare_result r;
  const int rc = orc_compare(in->n, in->la, in->La, in->lb, in->Lb, &r, ci, cj, cn, cap);
  put_i("rc", rc);
  if (rc == ORC_OK) {
    put_i("n", r.n), put_i("Ka", r.Ka), put_i("Kb", r.Kb), put_i("nnz", r.nnz);
    put_i("a11", r.a11), put_i("a10", r.a10), put_i("a01", r.a01), put_i("a00", r.a00), put_i("A", r.A);
    put_d("VI", r.VI), put_d("NMI", r.NMI), put_d("F", r.F), put_d("NVD", r.NVD);
    put_d("RI", r.RI), put_d("ARI", r.ARI), put_d("JI", r.JI);
    put_h("cell_i", ci, (size_t)r.nnz * 4), put_h("cell_j", cj, (size_t)r.nnz * 4);
    put_h("cell_n", cn, (size_t)r.nnz * 8);
  }
  free(ci), free(cj), free(cn);
}

int main(int argc, char** argv) {
  if (argc != 2) {
    fprintf(stderr, "usage: oracle_run INPUT\n");
    return 2;
  }
  host_input in;
  read_input(argv[1], &in);
  if (in.kind == 0) run_score(&in);
  else if (in.kind == 1) run_score_w(&in);
  else run_compare(&in);
  free_input(&in);
  return 0;
}
