// Host check of the library's two-chain band factor (factor.cpp, compiled into
// this program): on a randomly weighted grid Laplacian plus a small shift, the
// solve through the two chains, which meet at the separator, equals the solve
// through the single envelope factor; the separator comes out the same in both
// chains and every band position is owned by exactly one chain.
// Usage: twin_factor_check NX NY SEED; prints "m K s err sepdiff missing res".
#include <cstdio>
#include <cstdlib>
#include <map>
#include <random>

#include "factor.cpp"

using namespace spnet;

namespace {

// forward (columns from..to-1) or backward (all rows) sweep of one band stream
void sweep(int n, const std::vector<int32_t> &wf, const std::vector<double> &cv, const std::vector<int32_t> &wb,
           const std::vector<double> &rv, const std::vector<double> &inv, std::vector<double> &v, int from, int to,
           bool backward) {
  size_t off = 0;
  if (!backward) {
    for (int j = 0; j < n; ++j) {
      if (j >= from && j < to) {
        v[j] *= inv[j];
        for (int t = 0; t < wf[j]; ++t) v[j + 1 + t] -= cv[off + t] * v[j];
      }
      off += (size_t)wf[j];
    }
  } else {
    for (int s = 0; s < n; ++s) {
      const int i = n - 1 - s;
      v[i] *= inv[i];
      for (int t = 0; t < wb[s]; ++t) v[i - 1 - t] -= rv[off + t] * v[i];
      off += (size_t)wb[s];
    }
  }
}

}  // namespace

int main(int argc, char **argv) {
  if (argc < 4) return 2;
  const int nx = atoi(argv[1]), ny = atoi(argv[2]), seed = atoi(argv[3]);
  const int m = nx * ny;
  std::mt19937 rng((unsigned)seed);
  std::uniform_real_distribution<double> U(0.5, 1.5);
  std::vector<std::map<int, double>> rows((size_t)m);
  auto add = [&](int a, int b, double w) {
    rows[a][b] -= w;
    rows[b][a] -= w;
    rows[a][a] += w;
    rows[b][b] += w;
  };
  for (int y = 0; y < ny; ++y)
    for (int x = 0; x < nx; ++x) {
      const int i = y * nx + x;
      if (x + 1 < nx) add(i, i + 1, U(rng));
      if (y + 1 < ny) add(i, i + nx, U(rng));
      if (x + 1 < nx && y + 1 < ny && rng() % 3 == 0) add(i, i + nx + 1, U(rng));
      rows[i][i] += 1e-3;
    }
  System sys;
  sys.n = m;
  sys.rowptr.assign((size_t)m + 1, 0);
  for (int i = 0; i < m; ++i) {
    for (auto &e : rows[i]) {
      sys.col.push_back(e.first);
      sys.val.push_back(e.second);
    }
    sys.rowptr[i + 1] = (int64_t)sys.col.size();
  }
  std::vector<int32_t> dofs((size_t)m), where((size_t)m, -1);
  for (int i = 0; i < m; ++i) dofs[i] = i;
  StarFactor F;
  factor_star(sys, dofs.data(), m, where, F, 0);
  const int K = F.twin.K, s = F.twin.s, n = K + s;
  std::vector<double> b((size_t)m);
  for (auto &v : b) v = U(rng) - 1.0;
  // single chain
  std::vector<double> vp((size_t)m);
  for (int p = 0; p < m; ++p) vp[p] = b[F.perm[p]];
  sweep(m, F.width_fwd, F.colvals, F.width_bwd, F.rowvals, F.invdiag, vp, 0, m, false);
  sweep(m, F.width_fwd, F.colvals, F.width_bwd, F.rowvals, F.invdiag, vp, 0, m, true);
  double res = 0, bmax = 0;
  {
    std::vector<double> z((size_t)m);
    for (int p = 0; p < m; ++p) z[F.perm[p]] = vp[p];
    for (int i = 0; i < m; ++i) {
      double a = 0;
      for (int64_t q = sys.rowptr[i]; q < sys.rowptr[i + 1]; ++q) a += sys.val[q] * z[sys.col[q]];
      res = std::max(res, std::fabs(a - b[i]));
      bmax = std::max(bmax, std::fabs(b[i]));
    }
  }
  if (K == 0) {
    printf("%d 0 0 0 0 0 %.3e\n", m, res / bmax);
    return 0;
  }
  // two chains: forward apart, add the separator partial sums, finish the
  // separator in both, backward apart
  std::vector<double> v[2];
  for (int c = 0; c < 2; ++c) {
    v[c].assign((size_t)n, 0.0);
    for (int i = 0; i < n; ++i) {
      const int bp = F.twin.c[c].bpos[i];
      if (bp >= 0 && !(c == 1 && i >= K)) v[c][i] = b[F.perm[bp]];
    }
    const BandChain &C = F.twin.c[c];
    sweep(n, C.width_fwd, C.colvals, C.width_bwd, C.rowvals, C.invdiag, v[c], 0, K, false);
  }
  for (int i = K; i < n; ++i) {
    v[0][i] += v[1][i];
    v[1][i] = v[0][i];
  }
  for (int c = 0; c < 2; ++c) {
    const BandChain &C = F.twin.c[c];
    sweep(n, C.width_fwd, C.colvals, C.width_bwd, C.rowvals, C.invdiag, v[c], K, n, false);
    sweep(n, C.width_fwd, C.colvals, C.width_bwd, C.rowvals, C.invdiag, v[c], 0, n, true);
  }
  double err = 0, mx = 0, sepdiff = 0;
  std::vector<int> own((size_t)m, 0);
  for (int c = 0; c < 2; ++c)
    for (int i = 0; i < n; ++i) {
      const int bp = F.twin.c[c].bpos[i];
      if (bp < 0) continue;
      if (c == 1 && i >= K) {
        sepdiff = std::max(sepdiff, std::fabs(v[1][i] - v[0][i]));
        continue;
      }
      err = std::max(err, std::fabs(v[c][i] - vp[bp]));
      mx = std::max(mx, std::fabs(vp[bp]));
      own[bp]++;
    }
  int missing = 0;
  for (int p = 0; p < m; ++p) missing += own[p] != 1;
  printf("%d %d %d %.3e %.3e %d %.3e\n", m, K, s, err / mx, sepdiff, missing, res / bmax);
  return 0;
}
