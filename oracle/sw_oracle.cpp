// FP64 CPU oracle for the mW (Stillinger-Weber) hot path.
//
// TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the CPU
// baseline leg of the benchmark load this library.  It shares no code with the
// HIP engine and must never be used as a fallback for it.
//
// What it computes (Molinero & Moore, Sec. II.A, Eq. for E, phi2 and phi3, and
// the constants listed after them; mW values from Sec. II.D):
//
//   E   = sum_i sum_{j>i} phi2(r_ij) + sum_i sum_{j!=i} sum_{k>j, k!=i} phi3(r_ij, r_ik, theta_jik)
//   phi2(r)     = A eps [B (sig/r)^p - (sig/r)^q] exp(sig / (r - a sig))
//   phi3(r,s,t) = lam eps (cos t - cos t0)^2 exp(gam sig/(r - a sig)) exp(gam sig/(s - a sig))
//
// Every term is zero unless its distances are below a*sigma (the reduced
// cut-off of Sec. II.A).  Distances use the minimum image of a periodic
// orthorhombic box.  The vertex of theta_jik is the centre atom i (the angle
// between r_ij and r_ik), so each (centre, unordered pair of neighbours) is
// counted once.
//
// Forces are the analytic -grad E by the chain rule; the virial tensor is
// W_ab = sum over interactions of sum over legs d_a F_b (d = leg vector from
// the interaction's reference atom, F = force on the leg atom).  Velocity
// Verlet (kick-drift-kick) advances the state; the discrete adjoint of that
// map gives trajectory gradients.  Tangents (Hessian-vector products and
// parameter derivatives) come from forward-mode dual numbers running through
// the same force routine.
//
// Units: Angstrom, fs, kcal/mol, g/mol, K.  a[A/fs^2] = 4.184e-4 F/m.

#include <cmath>
#include <cstdint>
#include <cstring>
#include <vector>
#include <algorithm>
#include <type_traits>

namespace {

constexpr double kAcc = 4.184e-4;                  // (A/fs^2) / ((kcal/mol/A)/(g/mol))
constexpr double kBoltz = 8.314462618 / 4184.0;    // kcal/(mol K)

// ---------------------------------------------------------------- dual numbers
struct Dual {
  double v, d;
  Dual() : v(0), d(0) {}
  Dual(double x) : v(x), d(0) {}
  Dual(double x, double dx) : v(x), d(dx) {}
};
inline Dual operator+(Dual a, Dual b) { return {a.v + b.v, a.d + b.d}; }
inline Dual operator-(Dual a, Dual b) { return {a.v - b.v, a.d - b.d}; }
inline Dual operator-(Dual a) { return {-a.v, -a.d}; }
inline Dual operator*(Dual a, Dual b) { return {a.v * b.v, a.d * b.v + a.v * b.d}; }
inline Dual operator/(Dual a, Dual b) { return {a.v / b.v, (a.d * b.v - a.v * b.d) / (b.v * b.v)}; }
inline Dual& operator+=(Dual& a, Dual b) { a = a + b; return a; }
inline Dual& operator-=(Dual& a, Dual b) { a = a - b; return a; }
inline Dual sqrt(Dual a) { double s = std::sqrt(a.v); return {s, a.d / (2.0 * s)}; }
inline Dual exp(Dual a) { double e = std::exp(a.v); return {e, e * a.d}; }
inline Dual pow(Dual a, double p) {
  if (p == 0.0) return Dual(1.0);
  double y = std::pow(a.v, p);
  return {y, p * std::pow(a.v, p - 1.0) * a.d};
}
inline double val(double x) { return x; }
inline double val(const Dual& x) { return x.v; }
using std::sqrt; using std::exp; using std::pow;

// ---------------------------------------------------------------- parameters
// C layout of the parameter block: lambda, epsilon, sigma, A, B, p, q, gamma, a, cos_theta0.
template <class T>
struct Params {
  T lam, eps, sig, A, B; double p, q; T gam, a, cos0;
};

template <class T>
Params<T> make_params(const double* P, const double* Pdot) {
  auto mk = [&](int i) { return T(P[i]); };
  Params<T> out{mk(0), mk(1), mk(2), mk(3), mk(4), P[5], P[6], mk(7), mk(8), mk(9)};
  if constexpr (std::is_same<T, Dual>::value) {
    if (Pdot) {
      out.lam.d = Pdot[0]; out.eps.d = Pdot[1]; out.sig.d = Pdot[2]; out.A.d = Pdot[3];
      out.B.d = Pdot[4]; out.gam.d = Pdot[7]; out.a.d = Pdot[8]; out.cos0.d = Pdot[9];
    }
  }
  return out;
}

template <class T>
T phi2(T r, const Params<T>& P) {
  // Eq. phi2, zero at and beyond the cut-off a*sigma.
  T rc = P.a * P.sig;
  if (!(val(r) < val(rc))) return T(0.0);
  T sr = P.sig / r;
  return P.A * P.eps * (P.B * pow(sr, P.p) - pow(sr, P.q)) * exp(P.sig / (r - rc));
}

template <class T>
T leg(T r, const Params<T>& P) {
  // One radial factor of Eq. phi3: exp(gamma sigma / (r - a sigma)), zero beyond a*sigma.
  T rc = P.a * P.sig;
  if (!(val(r) < val(rc))) return T(0.0);
  return exp(P.gam * P.sig / (r - rc));
}

template <class T>
T phi3(T r, T s, T costh, const Params<T>& P) {
  T c = costh - P.cos0;
  return P.lam * P.eps * c * c * leg(r, P) * leg(s, P);
}

// ---------------------------------------------------------------- geometry
struct Box { double L[3]; };

// Minimum-image displacement x_j - x_i.  The image shift is a constant
// (integer multiple of the box edge), so tangents pass straight through.
template <class T>
void min_image(const T* xi, const T* xj, const Box& b, T d[3]) {
  for (int c = 0; c < 3; ++c) {
    T dc = xj[c] - xi[c];
    double s = b.L[c] * std::nearbyint(val(dc) / b.L[c]);
    d[c] = dc - T(s);
  }
}

// Neighbour pairs within rc, found by a plain cell list (cells of edge >= rc,
// 27-cell stencil) when every edge holds at least three cells, otherwise by
// testing all pairs.  Returns, for each atom, the sorted list of neighbours.
std::vector<std::vector<int>> neighbours(int n, const double* x, const Box& b, double rc) {
  std::vector<std::vector<int>> nb(n);
  int nc[3];
  for (int c = 0; c < 3; ++c) nc[c] = (int)std::floor(b.L[c] / rc);
  auto within = [&](int i, int j) {
    double d[3];
    min_image(x + 3 * i, x + 3 * j, b, d);
    return d[0] * d[0] + d[1] * d[1] + d[2] * d[2] < rc * rc;
  };
  if (nc[0] < 3 || nc[1] < 3 || nc[2] < 3) {
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j)
        if (j != i && within(i, j)) nb[i].push_back(j);
    return nb;
  }
  std::vector<std::vector<int>> cell((size_t)nc[0] * nc[1] * nc[2]);
  auto cidx = [&](int cx, int cy, int cz) {
    cx = (cx % nc[0] + nc[0]) % nc[0]; cy = (cy % nc[1] + nc[1]) % nc[1]; cz = (cz % nc[2] + nc[2]) % nc[2];
    return ((size_t)cx * nc[1] + cy) * nc[2] + cz;
  };
  std::vector<int> home(3 * (size_t)n);
  for (int i = 0; i < n; ++i) {
    int h[3];
    for (int c = 0; c < 3; ++c) {
      double u = x[3 * i + c] - b.L[c] * std::floor(x[3 * i + c] / b.L[c]);
      h[c] = std::min(nc[c] - 1, (int)(u / (b.L[c] / nc[c])));
      home[3 * i + c] = h[c];
    }
    cell[cidx(h[0], h[1], h[2])].push_back(i);
  }
  for (int i = 0; i < n; ++i) {
    for (int dx = -1; dx <= 1; ++dx)
      for (int dy = -1; dy <= 1; ++dy)
        for (int dz = -1; dz <= 1; ++dz)
          for (int j : cell[cidx(home[3 * i] + dx, home[3 * i + 1] + dy, home[3 * i + 2] + dz)])
            if (j != i && within(i, j)) nb[i].push_back(j);
    std::sort(nb[i].begin(), nb[i].end());
  }
  return nb;
}

// ---------------------------------------------------------------- forces
// Energy, forces and virial of Eq. E.  f, f3 are [n][3] (f3: three-body part
// only), e = {E2, E3}, w2, w3 = 3x3 virial tensors (row-major) of each term.
template <class T>
void evaluate(int n, const T* x, const Box& b, const Params<T>& P,
              T* f, T* f3, T* e, T* w2, T* w3) {
  std::vector<double> xv(3 * (size_t)n);
  for (size_t i = 0; i < xv.size(); ++i) xv[i] = val(x[i]);
  const double rc = val(P.a) * val(P.sig);
  auto nb = neighbours(n, xv.data(), b, rc);

  for (size_t i = 0; i < 3 * (size_t)n; ++i) { if (f) f[i] = T(0.0); if (f3) f3[i] = T(0.0); }
  T E2(0.0), E3(0.0);
  T W2[9], W3[9];
  for (int i = 0; i < 9; ++i) { W2[i] = T(0.0); W3[i] = T(0.0); }

  std::vector<T> d, r;   // per-neighbour displacement and distance of the current centre
  for (int i = 0; i < n; ++i) {
    const auto& J = nb[i];
    const int m = (int)J.size();
    d.assign(3 * (size_t)m, T(0.0));
    r.assign(m, T(0.0));
    for (int a = 0; a < m; ++a) {
      min_image(x + 3 * i, x + 3 * J[a], b, &d[3 * a]);
      r[a] = sqrt(d[3 * a] * d[3 * a] + d[3 * a + 1] * d[3 * a + 1] + d[3 * a + 2] * d[3 * a + 2]);
    }
    // Two-body term: the pair (i, j) once, with j > i.
    for (int a = 0; a < m; ++a) {
      const int j = J[a];
      if (j <= i) continue;
      // d(phi2)/dr by the chain rule of Eq. phi2:
      //   phi2 = A eps (B s^p - s^q) g,  s = sig/r, g = exp(sig/(r - rc))
      T rr = r[a], rcT = P.a * P.sig;
      if (!(val(rr) < val(rcT))) continue;
      T s = P.sig / rr;
      T poly = P.B * pow(s, P.p) - pow(s, P.q);
      T dpoly = (-(P.B * T(P.p) * pow(s, P.p)) + T(P.q) * pow(s, P.q)) / rr;   // d/dr
      T g = exp(P.sig / (rr - rcT));
      T dg = -g * P.sig / ((rr - rcT) * (rr - rcT));
      T ph = P.A * P.eps * poly * g;
      T dph = P.A * P.eps * (dpoly * g + poly * dg);
      E2 += ph;
      for (int c = 0; c < 3; ++c) {
        T fj = -dph * d[3 * a + c] / rr;          // force on j: -dphi/dr * d/r
        if (f) { f[3 * j + c] += fj; f[3 * i + c] -= fj; }
        for (int c2 = 0; c2 < 3; ++c2) W2[3 * c2 + c] += d[3 * a + c2] * fj;
      }
    }
    // Three-body term: centre i, neighbours j and k > j.
    for (int a = 0; a < m; ++a) {
      for (int bb = a + 1; bb < m; ++bb) {
        T rj = r[a], rk = r[bb];
        T rcT = P.a * P.sig;
        if (!(val(rj) < val(rcT)) || !(val(rk) < val(rcT))) continue;
        const T* dj = &d[3 * a];
        const T* dk = &d[3 * bb];
        T dot = dj[0] * dk[0] + dj[1] * dk[1] + dj[2] * dk[2];
        T cs = dot / (rj * rk);
        T ej = exp(P.gam * P.sig / (rj - rcT));
        T ek = exp(P.gam * P.sig / (rk - rcT));
        T dej = -ej * P.gam * P.sig / ((rj - rcT) * (rj - rcT));   // d ej / d rj
        T dek = -ek * P.gam * P.sig / ((rk - rcT) * (rk - rcT));
        T dc = cs - P.cos0;
        E3 += P.lam * P.eps * dc * dc * ej * ek;
        // gradient with respect to the leg vectors dj and dk
        T Fj[3], Fk[3];
        for (int c = 0; c < 3; ++c) {
          T dcs_dj = dk[c] / (rj * rk) - cs * dj[c] / (rj * rj);
          T dcs_dk = dj[c] / (rj * rk) - cs * dk[c] / (rk * rk);
          T gj = P.lam * P.eps * (T(2.0) * dc * dcs_dj * ej * ek + dc * dc * dej * (dj[c] / rj) * ek);
          T gk = P.lam * P.eps * (T(2.0) * dc * dcs_dk * ej * ek + dc * dc * ej * dek * (dk[c] / rk));
          Fj[c] = -gj;
          Fk[c] = -gk;
        }
        const int j = J[a], k = J[bb];
        for (int c = 0; c < 3; ++c) {
          if (f) { f[3 * j + c] += Fj[c]; f[3 * k + c] += Fk[c]; f[3 * i + c] -= Fj[c] + Fk[c]; }
          if (f3) { f3[3 * j + c] += Fj[c]; f3[3 * k + c] += Fk[c]; f3[3 * i + c] -= Fj[c] + Fk[c]; }
          for (int c2 = 0; c2 < 3; ++c2) W3[3 * c2 + c] += dj[c2] * Fj[c] + dk[c2] * Fk[c];
        }
      }
    }
  }
  if (e) { e[0] = E2; e[1] = E3; }
  for (int i = 0; i < 9; ++i) { if (w2) w2[i] = W2[i]; if (w3) w3[i] = W3[i]; }
}

// Brute force Eq. E over every index triple, O(N^3).
double brute_terms(int n, const double* x, const Box& b, const Params<double>& P, double* e3_out) {
  double E2 = 0.0, E3 = 0.0;
  auto dist = [&](int i, int j, double* d) {
    min_image(x + 3 * i, x + 3 * j, b, d);
    return std::sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
  };
  for (int i = 0; i < n; ++i)
    for (int j = i + 1; j < n; ++j) {
      double d[3];
      E2 += phi2(dist(i, j, d), P);
    }
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) {
      if (j == i) continue;
      double dj[3];
      double rj = dist(i, j, dj);
      if (!(rj < P.a * P.sig)) continue;
      for (int k = j + 1; k < n; ++k) {
        if (k == i) continue;
        double dk[3];
        double rk = dist(i, k, dk);
        if (!(rk < P.a * P.sig)) continue;
        double cs = (dj[0] * dk[0] + dj[1] * dk[1] + dj[2] * dk[2]) / (rj * rk);
        E3 += phi3(rj, rk, cs, P);
      }
    }
  *e3_out = E3;
  return E2;
}

Box make_box(const double* L) { Box b; for (int c = 0; c < 3; ++c) b.L[c] = L[c]; return b; }

double kinetic(int n, const double* v, double mass, double* kdiag) {
  double k[3] = {0, 0, 0};
  for (int i = 0; i < n; ++i)
    for (int c = 0; c < 3; ++c) k[c] += mass * v[3 * i + c] * v[3 * i + c] / kAcc;
  if (kdiag) for (int c = 0; c < 3; ++c) kdiag[c] = k[c];
  return 0.5 * (k[0] + k[1] + k[2]);
}

// Forces, energies and virial in plain doubles (value pass).
struct Eval {
  std::vector<double> f, f3;
  double e[2], w2[9], w3[9];
};
Eval eval_value(int n, const double* x, const Box& b, const double* P) {
  Eval ev;
  ev.f.assign(3 * (size_t)n, 0.0);
  ev.f3.assign(3 * (size_t)n, 0.0);
  Params<double> p = make_params<double>(P, nullptr);
  evaluate<double>(n, x, b, p, ev.f.data(), ev.f3.data(), ev.e, ev.w2, ev.w3);
  return ev;
}

// Tangent pass: positions moved along xdot, parameters along Pdot.
struct Tangent {
  std::vector<double> f, fdot, f3, f3dot;
  double e[2], edot[2], w2[9], w2dot[9], w3[9], w3dot[9];
};
Tangent eval_tangent(int n, const double* x, const double* xdot, const Box& b, const double* P,
                     const double* Pdot) {
  std::vector<Dual> xd(3 * (size_t)n), f(3 * (size_t)n), f3(3 * (size_t)n);
  for (size_t i = 0; i < xd.size(); ++i) xd[i] = Dual(x[i], xdot ? xdot[i] : 0.0);
  Params<Dual> p = make_params<Dual>(P, Pdot);
  Dual e[2], w2[9], w3[9];
  evaluate<Dual>(n, xd.data(), b, p, f.data(), f3.data(), e, w2, w3);
  Tangent t;
  t.f.resize(xd.size()); t.fdot.resize(xd.size()); t.f3.resize(xd.size()); t.f3dot.resize(xd.size());
  for (size_t i = 0; i < xd.size(); ++i) {
    t.f[i] = f[i].v; t.fdot[i] = f[i].d; t.f3[i] = f3[i].v; t.f3dot[i] = f3[i].d;
  }
  for (int k = 0; k < 2; ++k) { t.e[k] = e[k].v; t.edot[k] = e[k].d; }
  for (int k = 0; k < 9; ++k) { t.w2[k] = w2[k].v; t.w2dot[k] = w2[k].d; t.w3[k] = w3[k].v; t.w3dot[k] = w3[k].d; }
  return t;
}

void wrap_positions(int n, double* x, const Box& b) {
  for (int i = 0; i < n; ++i)
    for (int c = 0; c < 3; ++c) x[3 * i + c] -= b.L[c] * std::floor(x[3 * i + c] / b.L[c]);
}

}  // namespace

extern "C" {

// Single-term values for tests of the formulas themselves.
double ora_phi2(double r, const double* P) { return phi2<double>(r, make_params<double>(P, nullptr)); }
double ora_phi3(double r, double s, double costh, const double* P) {
  return phi3<double>(r, s, costh, make_params<double>(P, nullptr));
}

// Brute-force O(N^3) energy.  Returns 0, or -1 if the box is shorter than 2 a sigma.
int ora_energy_brute(int n, const double* x, const double* L, const double* P, double* e2, double* e3) {
  Box b = make_box(L);
  double rc = P[8] * P[2];
  for (int c = 0; c < 3; ++c) if (b.L[c] < 2.0 * rc) return -1;
  *e2 = brute_terms(n, x, b, make_params<double>(P, nullptr), e3);
  return 0;
}

// Energies e[2] = {E2, E3}, forces f[n][3], three-body forces f3[n][3]
// (may be NULL), virial tensors w2[9], w3[9] (row-major).
int ora_forces(int n, const double* x, const double* L, const double* P,
               double* f, double* f3, double* e, double* w2, double* w3) {
  Box b = make_box(L);
  double rc = P[8] * P[2];
  for (int c = 0; c < 3; ++c) if (b.L[c] < 2.0 * rc) return -1;
  Eval ev = eval_value(n, x, b, P);
  if (f) std::memcpy(f, ev.f.data(), sizeof(double) * 3 * n);
  if (f3) std::memcpy(f3, ev.f3.data(), sizeof(double) * 3 * n);
  if (e) { e[0] = ev.e[0]; e[1] = ev.e[1]; }
  if (w2) std::memcpy(w2, ev.w2, sizeof ev.w2);
  if (w3) std::memcpy(w3, ev.w3, sizeof ev.w3);
  return 0;
}

// Forward-mode tangent of everything ora_forces returns, with positions moved
// along xdot (may be NULL) and parameters along Pdot (may be NULL).  With
// Pdot = NULL, fdot = (dF/dx) xdot = -H xdot.
int ora_tangent(int n, const double* x, const double* xdot, const double* L, const double* P,
                const double* Pdot, double* f, double* fdot, double* f3, double* f3dot,
                double* e, double* edot, double* wdot_trace) {
  Box b = make_box(L);
  double rc = P[8] * P[2];
  for (int c = 0; c < 3; ++c) if (b.L[c] < 2.0 * rc) return -1;
  Tangent t = eval_tangent(n, x, xdot, b, P, Pdot);
  size_t bytes = sizeof(double) * 3 * n;
  if (f) std::memcpy(f, t.f.data(), bytes);
  if (fdot) std::memcpy(fdot, t.fdot.data(), bytes);
  if (f3) std::memcpy(f3, t.f3.data(), bytes);
  if (f3dot) std::memcpy(f3dot, t.f3dot.data(), bytes);
  if (e) { e[0] = t.e[0]; e[1] = t.e[1]; }
  if (edot) { edot[0] = t.edot[0]; edot[1] = t.edot[1]; }
  if (wdot_trace) {
    wdot_trace[0] = t.w2dot[0] + t.w2dot[4] + t.w2dot[8];
    wdot_trace[1] = t.w3dot[0] + t.w3dot[4] + t.w3dot[8];
  }
  return 0;
}

// Velocity Verlet (kick-drift-kick) in FP64.
//   v += dt/2 a(x);  x += dt v (wrapped into the box);  v += dt/2 a(x)
// then, for thermostat 1 (rescale) or 2 (Berendsen), v *= s with
//   s = sqrt(T0/T)  or  s = sqrt(1 + dt/tau (T0/T - 1)),
// T = 2 KE / ((3N - 3) k_B) measured on the full-step velocities.
// thermo[step][12] = E2, E3, KE (before scaling), W xx yy zz xy xz yz,
// K xx yy zz (K_aa = sum m v_a^2, kcal/mol), all at the end of the step.
// On return x, v, f hold the final state (f = F(x_final)).
int ora_vv(int n, double* x, double* v, double* f, const double* L, const double* P, double mass,
           double dt, int nsteps, int thermostat, double T0, double tau, double* thermo) {
  Box b = make_box(L);
  double rc = P[8] * P[2];
  for (int c = 0; c < 3; ++c) if (b.L[c] < 2.0 * rc) return -1;
  const double c_m = kAcc / mass;
  Eval ev = eval_value(n, x, b, P);
  for (int s = 0; s < nsteps; ++s) {
    for (int i = 0; i < 3 * n; ++i) v[i] += 0.5 * dt * c_m * ev.f[i];
    for (int i = 0; i < 3 * n; ++i) x[i] += dt * v[i];
    wrap_positions(n, x, b);
    ev = eval_value(n, x, b, P);
    for (int i = 0; i < 3 * n; ++i) v[i] += 0.5 * dt * c_m * ev.f[i];
    double kd[3];
    double ke = kinetic(n, v, mass, kd);
    if (thermo) {
      double* row = thermo + 12 * (size_t)s;
      row[0] = ev.e[0]; row[1] = ev.e[1]; row[2] = ke;
      double W[9];
      for (int k = 0; k < 9; ++k) W[k] = ev.w2[k] + ev.w3[k];
      row[3] = W[0]; row[4] = W[4]; row[5] = W[8]; row[6] = W[1]; row[7] = W[2]; row[8] = W[5];
      row[9] = kd[0]; row[10] = kd[1]; row[11] = kd[2];
    }
    if (thermostat == 1 || thermostat == 2) {
      double T = 2.0 * ke / ((3.0 * n - 3.0) * kBoltz);
      double scale = thermostat == 1 ? std::sqrt(T0 / T) : std::sqrt(1.0 + dt / tau * (T0 / T - 1.0));
      for (int i = 0; i < 3 * n; ++i) v[i] *= scale;
    }
  }
  if (f) std::memcpy(f, ev.f.data(), sizeof(double) * 3 * n);
  return 0;
}

// Virial trace W = sum over terms and legs of d . F (the configurational part
// of the pressure, P V = (2 KE + W) / 3).
double virial_trace(const Eval& ev) { return ev.w2[0] + ev.w2[4] + ev.w2[8] + ev.w3[0] + ev.w3[4] + ev.w3[8]; }

// Trajectory loss of the differentiable workload:
//   L = 1/(S+1) sum_{s=0..S} [aU U(x_s) + a3 U3(x_s) + aW W(x_s)] / N,
//   U = E2 + E3, U3 = E3, W the virial trace,
// over an NVE velocity-Verlet trajectory of S = nsteps steps from (x0, v0).
// x0 and v0 are left untouched; xS, vS (may be NULL) receive the final state.
double ora_traj_loss(int n, const double* x0, const double* v0, const double* L, const double* P,
                     double mass, double dt, int nsteps, double aU, double a3, double aW, double* xS, double* vS) {
  Box b = make_box(L);
  std::vector<double> x(x0, x0 + 3 * n), v(v0, v0 + 3 * n);
  const double c_m = kAcc / mass;
  const double norm = 1.0 / ((double)n * (nsteps + 1));
  Eval ev = eval_value(n, x.data(), b, P);
  double loss = (aU * (ev.e[0] + ev.e[1]) + a3 * ev.e[1] + aW * virial_trace(ev)) * norm;
  for (int s = 0; s < nsteps; ++s) {
    for (int i = 0; i < 3 * n; ++i) v[i] += 0.5 * dt * c_m * ev.f[i];
    for (int i = 0; i < 3 * n; ++i) x[i] += dt * v[i];
    wrap_positions(n, x.data(), b);
    ev = eval_value(n, x.data(), b, P);
    for (int i = 0; i < 3 * n; ++i) v[i] += 0.5 * dt * c_m * ev.f[i];
    loss += (aU * (ev.e[0] + ev.e[1]) + a3 * ev.e[1] + aW * virial_trace(ev)) * norm;
  }
  if (xS) std::memcpy(xS, x.data(), sizeof(double) * 3 * n);
  if (vS) std::memcpy(vS, v.data(), sizeof(double) * 3 * n);
  return loss;
}

// Discrete adjoint of the NVE velocity-Verlet map for the loss above, with
// optional terminal seeds xbar_S, vbar_S (dL_extra/dx_S, dL_extra/dv_S; may
// be NULL).  The whole trajectory is stored.  Reverse recursion, with
// a = c F / m and J = da/dx:
//   xb = xbar_S + dl_S/dx_S;  vb = vbar_S;  xb += h/2 J(x_S) vb
//   for n = S-1 .. 0:
//     vb += h xb
//     xb += w_n J(x_n) vb + dl_n/dx_n,   w_n = h (n > 0), h/2 (n = 0)
// and the parameter adjoint collects the same coefficients times vb . da/dtheta
// plus dl_n/dtheta.  J vb is the forward-mode tangent of the forces along vb
// (J is symmetric); da/dtheta comes from tangents in each parameter.  The
// virial term's gradient uses dU/dsigma = W/sigma (reduced form), hence
// dW/dx = sigma d(dU/dx)/dsigma = -sigma dF/dsigma, from the sigma tangent;
// its parameter derivatives are the tangents of the virial trace.
// Outputs: loss, xbar0[n][3], vbar0[n][3], thbar[3] = dL/d(lambda, epsilon, sigma).
int ora_adjoint(int n, const double* x0, const double* v0, const double* L, const double* P,
                double mass, double dt, int nsteps, double aU, double a3, double aW,
                const double* xbar_S, const double* vbar_S,
                double* loss_out, double* xbar0, double* vbar0, double* thbar) {
  Box b = make_box(L);
  double rc = P[8] * P[2];
  for (int c = 0; c < 3; ++c) if (b.L[c] < 2.0 * rc) return -1;
  const int S = nsteps;
  const size_t n3 = 3 * (size_t)n;
  const double c_m = kAcc / mass;
  const double norm = 1.0 / ((double)n * (S + 1));
  // forward, storing every frame
  std::vector<std::vector<double>> traj(S + 1);
  std::vector<double> x(x0, x0 + n3), v(v0, v0 + n3);
  traj[0] = x;
  Eval ev = eval_value(n, x.data(), b, P);
  double loss = (aU * (ev.e[0] + ev.e[1]) + a3 * ev.e[1] + aW * virial_trace(ev)) * norm;
  for (int s = 0; s < S; ++s) {
    for (size_t i = 0; i < n3; ++i) v[i] += 0.5 * dt * c_m * ev.f[i];
    for (size_t i = 0; i < n3; ++i) x[i] += dt * v[i];
    wrap_positions(n, x.data(), b);
    ev = eval_value(n, x.data(), b, P);
    for (size_t i = 0; i < n3; ++i) v[i] += 0.5 * dt * c_m * ev.f[i];
    loss += (aU * (ev.e[0] + ev.e[1]) + a3 * ev.e[1] + aW * virial_trace(ev)) * norm;
    traj[s + 1] = x;
  }
  *loss_out = loss;

  std::vector<double> xb(n3, 0.0), vb(n3, 0.0);
  double th[3] = {0.0, 0.0, 0.0};
  if (xbar_S) for (size_t i = 0; i < n3; ++i) xb[i] = xbar_S[i];
  if (vbar_S) for (size_t i = 0; i < n3; ++i) vb[i] = vbar_S[i];

  // dl/dx and dl/dtheta of frame s, plus coef * (J vb, vb . da/dtheta).
  auto frame = [&](int s, double coef) {
    const double* xs = traj[s].data();
    Tangent tp[3];
    for (int k = 0; k < 3; ++k) {           // tangents in lambda, epsilon, sigma
      double Pd[10] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
      Pd[k] = 1.0;
      tp[k] = eval_tangent(n, xs, nullptr, b, P, Pd);
    }
    for (int k = 0; k < 3; ++k) {           // uses vb before this frame's update of xb
      double vdF = 0.0;
      for (size_t i = 0; i < n3; ++i) vdF += vb[i] * tp[k].fdot[i];
      double wdot = 0.0;
      for (int c = 0; c < 9; c += 4) wdot += tp[k].w2dot[c] + tp[k].w3dot[c];
      th[k] += coef * c_m * vdF + (aU * (tp[k].edot[0] + tp[k].edot[1]) + a3 * tp[k].edot[1] + aW * wdot) * norm;
    }
    Tangent hv = eval_tangent(n, xs, vb.data(), b, P, nullptr);   // (dF/dx) vb
    const double sig = P[2];
    for (size_t i = 0; i < n3; ++i)
      xb[i] += coef * c_m * hv.fdot[i] - (aU * hv.f[i] + a3 * hv.f3[i]) * norm - aW * sig * tp[2].fdot[i] * norm;
  };
  frame(S, 0.5 * dt);
  for (int s = S - 1; s >= 0; --s) {
    for (size_t i = 0; i < n3; ++i) vb[i] += dt * xb[i];
    frame(s, s > 0 ? dt : 0.5 * dt);
  }
  std::memcpy(xbar0, xb.data(), sizeof(double) * n3);
  std::memcpy(vbar0, vb.data(), sizeof(double) * n3);
  for (int k = 0; k < 3; ++k) thbar[k] = th[k];
  return 0;
}

// Isothermal-isobaric dynamics (the Nose-Hoover thermostat and barostat of
// Sec. II.B, relaxation times tau_T and tau_P, pressure p), read as the
// isotropic Martyna-Tobias-Klein equations with Nose-Hoover chains of length M
// on the particles (xi) and on the barostat (eta):
//   dr/dt = v + v_e r,          dv/dt = a(r) - (1 + 3/Nf) v_e v - vxi_1 v
//   dL/dt = v_e L (each edge),  dv_e/dt = [(1 + 3/Nf) sum m v^2 + W - 3 p V] / Wb - veta_1 v_e
//   chains: dvxi_1/dt = (sum m v^2 - Nf kT)/Q_1 - vxi_2 vxi_1, ..., same for eta
//           with Wb v_e^2 in place of sum m v^2 and 1 in place of Nf,
// Nf = 3N - 3, W = virial trace, masses Q_1 = Nf kT tau_T^2, Q_k = kT tau_T^2,
// Wb = (Nf + 3) kT tau_P^2, Q'_k = kT tau_P^2.  Conserved:
//   H' = KE + U + p V + Wb v_e^2/2 + sum_k Q_k vxi_k^2/2 + Nf kT xi_1 + kT sum_{k>1} xi_k
//        + sum_k Q'_k veta_k^2/2 + kT sum_k eta_k.
// One step of length dt = 2h is the symmetric splitting
//   chain(eta, h) chain(xi, h) baro(h) kick(h) drift(2h) kick(h) baro(h) chain(xi, h) chain(eta, h)
// with the exact flows kick: v <- v e^{-c h} + h a e^{-c h/2} sinhc(c h/2), c = (1 + 3/Nf) v_e;
// drift: r <- r e^{v_e dt} + v dt e^{v_e dt/2} sinhc(v_e dt/2), L <- L e^{v_e dt};
// baro: v_e += h [(1 + 3/Nf) sum m v^2 + W - 3 p V] / Wb; and a chain half step
// of one Suzuki-Yoshida stage.  Pressure p in kcal/mol/A^3.
// tauP <= 0 removes the barostat (fixed box, Nose-Hoover NVT, v_e = 0).
// state: [0] v_e, [1..4] xi, [5..8] vxi, [9..12] eta, [13..16] veta (chain M <= 4).
// rows (may be NULL): per step, after the step: V, P_int (kcal/mol/A^3), T, U, KE,
// p V, the extended energies, H', and the pressure tensor diagonal
// P_aa = (sum m v_a^2 + W_aa) / V.
namespace {
double sinhc(double x) { return std::fabs(x) < 1e-4 ? 1.0 + x * x / 6.0 : std::sinh(x) / x; }

// One chain half step of length h on a subsystem with kinetic term k2 (twice
// its kinetic energy) and nf degrees of freedom; returns the velocity scale.
double chain_half(double h, double& k2, double nf, double kT, const double* Q, double* xi, double* vxi, int M) {
  auto G = [&](int k) { return k == 0 ? (k2 - nf * kT) / Q[0] : (Q[k - 1] * vxi[k - 1] * vxi[k - 1] - kT) / Q[k]; };
  vxi[M - 1] += 0.5 * h * G(M - 1);
  for (int k = M - 2; k >= 0; --k) {
    const double e = std::exp(-0.25 * h * vxi[k + 1]);
    vxi[k] = (vxi[k] * e + 0.5 * h * G(k)) * e;
  }
  const double s = std::exp(-h * vxi[0]);
  k2 *= s * s;
  for (int k = 0; k < M; ++k) xi[k] += h * vxi[k];
  for (int k = 0; k < M - 1; ++k) {
    const double e = std::exp(-0.25 * h * vxi[k + 1]);
    vxi[k] = (vxi[k] * e + 0.5 * h * G(k)) * e;
  }
  vxi[M - 1] += 0.5 * h * G(M - 1);
  return s;
}
}  // namespace

int ora_npt(int n, double* x, double* v, double* L, const double* P, double mass, double dt, int nsteps,
            double T0, double p_ext, double tauT, double tauP, int M, double* state, double* rows) {
  if (M < 1 || M > 4 || n < 2) return -2;
  const double rc = P[8] * P[2];
  for (int c = 0; c < 3; ++c) if (L[c] < 2.0 * rc) return -1;
  const double c_m = kAcc / mass, h = 0.5 * dt;
  const double nf = 3.0 * n - 3.0, kT = kBoltz * T0, alpha = 1.0 + 3.0 / nf;
  double Q[4], Qb[4];
  for (int k = 0; k < 4; ++k) {
    Q[k] = (k == 0 ? nf : 1.0) * kT * tauT * tauT;
    Qb[k] = kT * tauP * tauP;
  }
  const bool baro = tauP > 0.0;
  if (!baro) p_ext = 0.0;
  const double Wb = (nf + 3.0) * kT * tauP * tauP;
  double& ve = state[0];
  double *xi = state + 1, *vxi = state + 5, *eta = state + 9, *veta = state + 13;
  Box b = make_box(L);
  Eval ev = eval_value(n, x, b, P);
  auto vir = [&]() { return ev.w2[0] + ev.w2[4] + ev.w2[8] + ev.w3[0] + ev.w3[4] + ev.w3[8]; };
  auto k2_of = [&]() { return 2.0 * kinetic(n, v, mass, nullptr); };
  auto barostat = [&](double k2) {
    if (!baro) return;
    const double V = b.L[0] * b.L[1] * b.L[2];
    ve += h * (alpha * k2 + vir() - 3.0 * p_ext * V) / Wb;
  };
  auto kick = [&]() {
    const double c = alpha * ve;
    const double ea = std::exp(-c * h), eb = h * c_m * std::exp(-0.5 * c * h) * sinhc(0.5 * c * h);
    for (int i = 0; i < 3 * n; ++i) v[i] = v[i] * ea + eb * ev.f[i];
  };
  auto chains = [&](double& k2, bool first) {
    double kb = Wb * ve * ve;
    if (first) {
      if (baro) ve *= chain_half(h, kb, 1.0, kT, Qb, eta, veta, M);
      const double s = chain_half(h, k2, nf, kT, Q, xi, vxi, M);
      for (int i = 0; i < 3 * n; ++i) v[i] *= s;
    } else {
      const double s = chain_half(h, k2, nf, kT, Q, xi, vxi, M);
      for (int i = 0; i < 3 * n; ++i) v[i] *= s;
      kb = Wb * ve * ve;
      if (baro) ve *= chain_half(h, kb, 1.0, kT, Qb, eta, veta, M);
    }
  };
  for (int s = 0; s < nsteps; ++s) {
    double k2 = k2_of();
    chains(k2, true);
    barostat(k2_of());
    kick();
    const double g = std::exp(ve * dt), d = dt * std::exp(0.5 * ve * dt) * sinhc(0.5 * ve * dt);
    for (int i = 0; i < 3 * n; ++i) x[i] = x[i] * g + v[i] * d;
    for (int c = 0; c < 3; ++c) b.L[c] *= g;
    wrap_positions(n, x, b);
    ev = eval_value(n, x, b, P);
    kick();
    barostat(k2_of());
    k2 = k2_of();
    chains(k2, false);
    if (rows) {
      const double V = b.L[0] * b.L[1] * b.L[2];
      double kd[3];
      const double ke = kinetic(n, v, mass, kd), U = ev.e[0] + ev.e[1];
      double ext = baro ? 0.5 * Wb * ve * ve : 0.0;
      for (int k = 0; k < M; ++k) {
        ext += 0.5 * Q[k] * vxi[k] * vxi[k] + (k == 0 ? nf : 1.0) * kT * xi[k];
        if (baro) ext += 0.5 * Qb[k] * veta[k] * veta[k] + kT * eta[k];
      }
      double* row = rows + 11 * (size_t)s;
      row[0] = V; row[1] = (2.0 * ke + vir()) / (3.0 * V); row[2] = 2.0 * ke / (nf * kBoltz); row[3] = U;
      row[4] = ke; row[5] = p_ext * V; row[6] = ext; row[7] = ke + U + p_ext * V + ext;
      for (int c = 0; c < 3; ++c) row[8 + c] = (kd[c] + ev.w2[4 * c] + ev.w3[4 * c]) / V;
    }
  }
  for (int c = 0; c < 3; ++c) L[c] = b.L[c];
  return 0;
}

// Number of neighbours within rc of each atom (for list-capacity checks).
int ora_neighbour_counts(int n, const double* x, const double* L, double rc, int* counts) {
  Box b = make_box(L);
  for (int c = 0; c < 3; ++c) if (b.L[c] < 2.0 * rc) return -1;
  auto nb = neighbours(n, x, b, rc);
  for (int i = 0; i < n; ++i) counts[i] = (int)nb[i].size();
  return 0;
}

// Neighbour sets within rc as CSR: offsets[n+1], idx[offsets[n]] (each row
// sorted).  Call with idx = NULL to get offsets only.
int ora_neighbour_lists(int n, const double* x, const double* L, double rc, long long* offsets, int* idx) {
  Box b = make_box(L);
  for (int c = 0; c < 3; ++c) if (b.L[c] < 2.0 * rc) return -1;
  auto nb = neighbours(n, x, b, rc);
  offsets[0] = 0;
  for (int i = 0; i < n; ++i) offsets[i + 1] = offsets[i] + (long long)nb[i].size();
  if (idx)
    for (int i = 0; i < n; ++i)
      for (size_t k = 0; k < nb[i].size(); ++k) idx[offsets[i] + (long long)k] = nb[i][k];
  return 0;
}

}  // extern "C"
