/* Runs the pthreads CPU scorer once on a score input file (host_input.h) with the given
 * thread count and prints its results exactly.  Built with the thread sanitizer, and
 * with the address and undefined-behaviour sanitizers, by tests/test_host_sanitized.py,
 * which compares the printout with the oracle's results. */
#include "cq_cpu_pthreads.c"
#include "host_input.h"

int main(int argc, char** argv) {
  if (argc != 3) {
    fprintf(stderr, "usage: cpubase_run INPUT THREADS\n");
    return 2;
  }
  host_input in;
  read_input(argv[1], &in);
  cpu_score_result r;
  const int rc = cpu_score(in.n, in.rp, in.ci, in.lab, in.L, atoi(argv[2]), &r);
  put_i("rc", rc);
  if (rc == 0) {
    put_i("n", r.n), put_i("m", r.m), put_i("K", r.K), put_i("num_pairs", r.num_pairs);
    put_i("sum_ein", r.sum_ein), put_i("sum_eout", r.sum_eout);
    put_d("Q", r.Q), put_d("Qds", r.Qds), put_d("split_penalty", r.split_penalty);
    put_d("mean_intra_edges", r.mean_intra_edges), put_d("mean_intra_density", r.mean_intra_density);
    put_d("mean_contraction", r.mean_contraction), put_d("mean_inter_edges", r.mean_inter_edges);
    put_d("mean_expansion", r.mean_expansion), put_d("mean_conductance", r.mean_conductance);
  }
  free_input(&in);
  return 0;
}
