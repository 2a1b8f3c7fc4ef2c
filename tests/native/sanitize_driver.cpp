// Runs the native host code of the test infrastructure -- the synthetic-graph
// generators and the oracle's C passes (CSR build, forward levels,
// back-accumulation, walk pairs) -- on small graphs, so that a build with
// AddressSanitizer and UndefinedBehaviorSanitizer checks every access.
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <utility>
#include <vector>

extern "C" {
int gg_rmat(int32_t n, int64_t m, double a, double b, double c, double d, uint64_t seed, int32_t* src, int32_t* dst);
int gg_chung_lu(int32_t n, int64_t m, double gamma, uint64_t seed, int32_t* src, int32_t* dst);
int oracle_in_csr(int64_t n, int64_t m, const int32_t* src, const int32_t* dst, int64_t* din, double* inv_din,
                  int64_t* in_off, int32_t* in_idx);
void oracle_out_off(int64_t n, int64_t m, const int32_t* src, int64_t* out_off);
int oracle_forward(int64_t n, const int64_t* out_off, const int32_t* out_idx, const double* inv_din, int64_t u,
                   double c, int L, double* levels, double* pi);
int oracle_backward(int64_t n, const int64_t* in_off, const int32_t* in_idx, const double* inv_din,
                    const double* levels, int L, const double* D, double c, double* s);
int oracle_walk_counts(int64_t n, const int64_t* in_off, const int32_t* in_idx, const uint64_t* r_begin,
                       const uint64_t* r_end, const int32_t* nonstop, uint64_t seed, double c, uint64_t* M,
                       int threads);
}

static int run(const char* name, int32_t n, std::vector<int32_t> src, std::vector<int32_t> dst) {
  const int64_t m = (int64_t)src.size();
  std::vector<std::pair<int32_t, int32_t>> e(m);
  for (int64_t i = 0; i < m; ++i) e[i] = {src[i], dst[i]};
  std::sort(e.begin(), e.end());
  for (int64_t i = 0; i < m; ++i) {
    src[i] = e[i].first;
    dst[i] = e[i].second;
  }
  std::vector<int64_t> din(n), in_off(n + 1), out_off(n + 1);
  std::vector<double> inv_din(n);
  std::vector<int32_t> in_idx(m);
  if (oracle_in_csr(n, m, src.data(), dst.data(), din.data(), inv_din.data(), in_off.data(), in_idx.data()) != 0)
    return 1;
  oracle_out_off(n, m, src.data(), out_off.data());
  const double c = 0.6;
  const int L = 12;
  std::vector<double> levels((size_t)(L + 1) * n), pi(n), D(n, 0.8), s(n);
  int64_t u = 0;
  for (int32_t k = 0; k < n; ++k)
    if (din[k] > din[u]) u = k;
  if (oracle_forward(n, out_off.data(), dst.data(), inv_din.data(), u, c, L, levels.data(), pi.data()) != 0) return 2;
  if (oracle_backward(n, in_off.data(), in_idx.data(), inv_din.data(), levels.data(), L, D.data(), c, s.data()) != 0)
    return 3;
  // a few hundred pairs per node, and a non-stop level on the source
  std::vector<uint64_t> r_end(n), M(n);
  std::vector<int32_t> nonstop(n, 0);
  for (int32_t k = 0; k < n; ++k) r_end[k] = (uint64_t)(200.0 * std::sqrt((double)din[k]));
  nonstop[u] = 2;
  if (oracle_walk_counts(n, in_off.data(), in_idx.data(), nullptr, r_end.data(), nullptr, 7, c, M.data(), 2) != 0)
    return 4;
  if (oracle_walk_counts(n, in_off.data(), in_idx.data(), nullptr, r_end.data(), nonstop.data(), 7, c, M.data(), 2))
    return 5;
  uint64_t meets = 0;
  for (int32_t k = 0; k < n; ++k) meets += M[k];
  std::printf("%s: n=%d m=%lld s(u,u)=%.6f meets=%llu\n", name, n, (long long)m, s[u], (unsigned long long)meets);
  return 0;
}

int main() {
  {
    const int32_t n = 4096;
    const int64_t m = 40000;
    std::vector<int32_t> src(m), dst(m);
    if (gg_rmat(n, m, 0.57, 0.19, 0.19, 0.05, 11, src.data(), dst.data()) != 0) return 10;
    if (int r = run("rmat", n, src, dst)) return r;
  }
  {
    const int32_t n = 2000;
    const int64_t m = 20000;
    std::vector<int32_t> src(m), dst(m);
    if (gg_chung_lu(n, m, 2.1, 12, src.data(), dst.data()) != 0) return 20;
    if (int r = run("chung_lu", n, src, dst)) return 20 + r;
  }
  std::printf("ok\n");
  return 0;
}
