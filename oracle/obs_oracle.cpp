// FP64 CPU oracle for the structural observables of Sec. II.C of the mW
// paper: the pair distribution (g(r), as a histogram of pair distances), the
// angular distribution of each molecule's n_c closest neighbours (P(theta)),
// and the unwrapped displacement behind the Einstein relation for D.
//
// TEST INFRASTRUCTURE ONLY (see __init__.py).  Plain loops over all pairs.
//
// Coordinates follow the engine's documented convention: each coordinate is
// held as a 32-bit unsigned fraction of its box edge,
//   u = floor(frac(x / L) * 2^32),   frac(y) = y - floor(y),
// and the minimum-image difference of two atoms is the two's-complement value
// of u_j - u_i times L / 2^32.  Distances and angles are then formed with
// single IEEE double operations in a fixed order (this file is compiled
// without floating-point contraction), so a histogram bin is an exact
// function of the inputs and of the caller's bin edges.
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <vector>

namespace {

uint32_t quantize(double x, double L) {
  double fr = x * (1.0 / L);
  fr -= std::floor(fr);
  return (uint32_t)(uint64_t)(fr * 4294967296.0);   // 2^32 wraps to 0
}

struct Frac {
  std::vector<uint32_t> u;   // [n][3]
  double sc[3];              // L / 2^32
};

Frac to_frac(int n, const double* x, const double* L) {
  Frac f;
  f.u.resize((size_t)3 * n);
  for (int c = 0; c < 3; ++c) f.sc[c] = L[c] / 4294967296.0;
  for (int i = 0; i < n; ++i)
    for (int c = 0; c < 3; ++c) f.u[(size_t)3 * i + c] = quantize(x[(size_t)3 * i + c], L[c]);
  return f;
}

// minimum-image difference r_j - r_i
void diff(const Frac& f, int i, int j, double d[3]) {
  for (int c = 0; c < 3; ++c) {
    const uint32_t a = f.u[(size_t)3 * i + c], b = f.u[(size_t)3 * j + c];
    d[c] = (double)(int32_t)(b - a) * f.sc[c];
  }
}

double norm2(const double d[3]) { return (d[0] * d[0] + d[1] * d[1]) + d[2] * d[2]; }

}  // namespace

extern "C" {

// Quantised coordinates of n atoms (for tests of the convention itself).
void ora_quantize(int n, const double* x, const double* L, uint32_t* u) {
  for (int i = 0; i < n; ++i)
    for (int c = 0; c < 3; ++c) u[(size_t)3 * i + c] = quantize(x[(size_t)3 * i + c], L[c]);
}

// Pair-distance histogram: ordered pairs (i, j), j != i, with
// e[0] <= r^2 < e[nb]; the bin is the number of interior edges e[1..nb-1]
// that are <= r^2.  g(r) follows by dividing by N^2/V times each shell's
// volume (Sec. II.C).
void ora_rdf(int n, const double* x, const double* L, int nb, const double* e, uint64_t* counts) {
  const Frac f = to_frac(n, x, L);
  for (int k = 0; k < nb; ++k) counts[k] = 0;
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) {
      if (j == i) continue;
      double d[3];
      diff(f, i, j, d);
      const double r2 = norm2(d);
      if (!(r2 >= e[0] && r2 < e[nb])) continue;
      int k = 0;
      for (int m = 1; m < nb; ++m) k += e[m] <= r2;
      ++counts[k];
    }
}

// Angular distribution: for every centre k, its neighbours j with
// r^2 < rs2 ordered by (r^2, index); the first n_near of them, and every
// unordered pair (a, b) of those gives cos(theta_akb) = (d_a . d_b) /
// sqrt(r_a^2 r_b^2).  The bin is the number of interior edges c[1..nb-1]
// (descending cosines, i.e. ascending angles) that are >= cos.  Centres with
// fewer than n_near neighbours inside rs are counted in *n_short and skipped.
void ora_adf(int n, const double* x, const double* L, int n_near, double rs2, int nb, const double* c,
             uint64_t* counts, long long* n_short) {
  const Frac f = to_frac(n, x, L);
  for (int k = 0; k < nb; ++k) counts[k] = 0;
  *n_short = 0;
  struct Nb {
    double r2;
    int j;
    double d[3];
  };
  std::vector<Nb> nbrs;
  for (int k = 0; k < n; ++k) {
    nbrs.clear();
    for (int j = 0; j < n; ++j) {
      if (j == k) continue;
      Nb b;
      diff(f, k, j, b.d);
      b.r2 = norm2(b.d);
      b.j = j;
      if (b.r2 < rs2) nbrs.push_back(b);
    }
    if ((int)nbrs.size() < n_near) {
      ++*n_short;
      continue;
    }
    std::sort(nbrs.begin(), nbrs.end(),
              [](const Nb& p, const Nb& q) { return p.r2 < q.r2 || (p.r2 == q.r2 && p.j < q.j); });
    for (int a = 0; a < n_near; ++a)
      for (int b = a + 1; b < n_near; ++b) {
        const double* da = nbrs[a].d;
        const double* db = nbrs[b].d;
        const double dot = (da[0] * db[0] + da[1] * db[1]) + da[2] * db[2];
        const double cs = dot / std::sqrt(nbrs[a].r2 * nbrs[b].r2);
        int m = 0;
        for (int t = 1; t < nb; ++t) m += c[t] >= cs;
        ++counts[m];
      }
  }
}

}  // extern "C"
