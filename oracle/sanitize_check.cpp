// TEST INFRASTRUCTURE ONLY: a driver that calls every C entry point of the
// oracle on tiny lattices with random inputs, for a build of the oracle with
// the address and undefined-behaviour sanitizers (tests/test_oracle_sanitizers.py).
// It checks memory safety, not values: the value checks live in the tests.
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <random>
#include <vector>

extern "C" {
int oracle_num_threads(void);
int oracle_site_maps(const int *L, int parity, int32_t *lex_of_cb, int32_t *nbr);
int oracle_block_of_site(const int *L, const int *nblk, int32_t *block_of_lex);
int oracle_op5_matrix(int Ls, const double *p, int which, double *mat);
int oracle_hop_full(const int *L, int Ls, const double *p, const double *U, double *out, const double *in, int sg);
int oracle_D_full(const int *L, int Ls, const double *p, const double *U, double *out, const double *in);
int oracle_dslash_eo(const int *L, int Ls, const double *p, const double *U, double *out, const double *in,
                     int out_parity, int dagger);
int oracle_op5(const int *L, int Ls, const double *p, double *out, const double *in, int parity, int which);
int oracle_dpc(const int *L, int Ls, const double *p, const double *U, double *out, const double *in, int parity,
               int dagger);
int oracle_mdagm(const int *L, int Ls, const double *p, const double *U, double *out, const double *in);
int oracle_prepare_rhs(const int *L, int Ls, const double *p, const double *U, double *b_even, double *phihat_even,
                       const double *phi_lex);
int oracle_reconstruct(const int *L, int Ls, const double *p, const double *U, double *psi_lex,
                       const double *psi_even, const double *phi_lex);
int oracle_block_op(const int *L, int Ls, const double *p, const double *U, double *out, const double *in,
                    const int *nblk, int block, int truncated);
int oracle_local_block_cg(const int *L, int Ls, const double *p, const double *U, double *z, const double *r,
                          const int *nblk, int k, int truncated, double inner_tol, int sweeps);
int oracle_solve(const int *L, int Ls, const double *p, const double *U, double *x, const double *b,
                 const int *nblk, int k, int truncated, double tol, int maxiter, int reliable, double *out_stats,
                 double *hist, int hist_len, double inner_tol, int sweeps, int flexible);
}

namespace {
int failures = 0;
void expect(bool ok, const char *what) {
  if (!ok) {
    std::printf("FAILED: %s\n", what);
    ++failures;
  }
}
std::vector<double> randv(size_t n, std::mt19937_64 &g) {
  std::normal_distribution<double> d;
  std::vector<double> v(n);
  for (auto &x : v) x = d(g);
  return v;
}
}  // namespace

int main() {
  std::mt19937_64 g(7);
  const int L[4] = {4, 2, 2, 6};
  const int Ls = 4, V = 4 * 2 * 2 * 6, Vh = V / 2;
  const double p[5] = {1.8, 0.05, 1.5, 0.5, -1.0};
  const size_t full = (size_t)V * Ls * 24, half = (size_t)Vh * Ls * 24;
  std::vector<double> U = randv((size_t)V * 4 * 18, g);  // memory checks only: any link values
  std::vector<double> in_full = randv(full, g), out_full(full), in_half = randv(half, g), out_half(half);
  std::vector<int32_t> lex(Vh), nbr((size_t)Vh * 8), blk(V);
  const int nblk[4] = {2, 1, 1, 2};
  expect(oracle_num_threads() >= 1, "threads");
  for (int par = 0; par < 2; ++par) expect(oracle_site_maps(L, par, lex.data(), nbr.data()) == 0, "site_maps");
  expect(oracle_block_of_site(L, nblk, blk.data()) == 0, "block_of_site");
  std::vector<double> mat((size_t)(4 * Ls) * (4 * Ls) * 2);
  for (int w = 0; w < 7; ++w) expect(oracle_op5_matrix(Ls, p, w, mat.data()) == 0, "op5_matrix");
  expect(oracle_op5_matrix(Ls, p, 99, mat.data()) == -1, "op5_matrix rejects a bad index");
  for (int sg : {1, -1}) expect(oracle_hop_full(L, Ls, p, U.data(), out_full.data(), in_full.data(), sg) == 0, "hop");
  expect(oracle_D_full(L, Ls, p, U.data(), out_full.data(), in_full.data()) == 0, "D_full");
  for (int par = 0; par < 2; ++par)
    for (int dag = 0; dag < 2; ++dag) {
      expect(oracle_dslash_eo(L, Ls, p, U.data(), out_half.data(), in_half.data(), par, dag) == 0, "dslash_eo");
      expect(oracle_dpc(L, Ls, p, U.data(), out_half.data(), in_half.data(), par, dag) == 0, "dpc");
    }
  for (int w = 0; w < 7; ++w) expect(oracle_op5(L, Ls, p, out_half.data(), in_half.data(), 1, w) == 0, "op5");
  expect(oracle_mdagm(L, Ls, p, U.data(), out_half.data(), in_half.data()) == 0, "mdagm");
  std::vector<double> b(half), ph(half), psi(full);
  expect(oracle_prepare_rhs(L, Ls, p, U.data(), b.data(), ph.data(), in_full.data()) == 0, "prepare_rhs");
  expect(oracle_reconstruct(L, Ls, p, U.data(), psi.data(), in_half.data(), in_full.data()) == 0, "reconstruct");
  for (int blkid = 0; blkid < 4; ++blkid)
    for (int tr = 0; tr < 2; ++tr)
      expect(oracle_block_op(L, Ls, p, U.data(), out_half.data(), in_half.data(), nblk, blkid, tr) == 0, "block_op");
  expect(oracle_block_op(L, Ls, p, U.data(), out_half.data(), in_half.data(), nblk, 4, 0) == -1, "block range");
  expect(oracle_local_block_cg(L, Ls, p, U.data(), out_half.data(), in_half.data(), nblk, 3, 0, 0.0, 1) == 0, "lbcg");
  expect(oracle_local_block_cg(L, Ls, p, U.data(), out_half.data(), in_half.data(), nblk, 4, 1, 0.1, 2) == 0,
         "lbcg with stopping and sweeps");
  double stats[3], hist[8];
  std::vector<double> x(half, 0.0);
  expect(oracle_solve(L, Ls, p, U.data(), x.data(), in_half.data(), nullptr, 0, 0, 1e-6, 50, 10, stats, hist, 8,
                      0.0, 1, 0) == 0, "solve (CG)");
  for (int flex = 0; flex < 2; ++flex) {
    std::fill(x.begin(), x.end(), 0.0);
    expect(oracle_solve(L, Ls, p, U.data(), x.data(), in_half.data(), nblk, 2, 0, 1e-6, 30, 5, stats, hist, 8, 0.0,
                        1, flex) == 0, "solve (MSPCG)");
  }
  for (double v : x) expect(std::isfinite(v), "finite solution");
  std::printf(failures ? "sanitize check: %d failures\n" : "sanitize check: ok\n", failures);
  return failures ? 1 : 0;
}
