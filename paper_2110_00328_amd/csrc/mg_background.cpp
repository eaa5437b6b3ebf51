// Coupled-quintessence background (Sec. 4.3, background cosmology solver):
// the homogeneous field phi-bar(a), H(a), dH/dt and the lambda of
// eq:csf_param_lambda that makes H(a=1) = H0.  Host code in FP64: a scalar
// ODE integrated once per model, whose table the field solver and the
// particle kick read.
//
// Time variable N = ln a; E = (aH/H0)^2; D = (d(aH)/dtau)/H0^2;
// P = phi-bar, Q = dP/dN.  The code-unit equations after
// eq:csf_background_Raychaudhuri, with the potential coefficient written
// "lambda" there taken as lambda^2/3 (V/(3 M_Pl^2) in the Friedmann equation
// with V = M_Pl^2 H0^2 lambda^2 phi^-alpha), which is what makes the two
// forms and eq:csf_background_eom_codeunit consistent with the potential
// force alpha lambda^2 of eq:csf_eom_code:
//   E (1 - Q^2/6) = Om_r e^-2N + Om_m e^-N e^{beta P} + (lambda^2/3) e^2N P^-alpha
//   D = -(1/3) Q^2 E + (lambda^2/3) e^2N P^-alpha - Om_r e^-2N - (1/2) Om_m e^-N e^{beta P}
//   E dQ/dN = alpha lambda^2 e^2N P^-(1+alpha) - 3 beta Om_m e^-N e^{beta P} - (2E + D) Q
//
// The paper integrates with a fifth/sixth-order Runge-Kutta pair; this uses
// the Dormand-Prince 5(4) pair (Dormand & Prince 1980) with local error
// control, stepping exactly onto every table node.
#include <cmath>
#include <cstring>

#include "mggpu.h"

namespace {

constexpr double kPi = 3.14159265358979323846;

struct Model {
  double om, orad, alpha, beta, lam2;
};

// E, D and dQ/dN at (N, P, Q); false when the state left the domain
// (P <= 0, Q^2 >= 6 or a non-finite value)
bool eval(const Model& m, double N, double P, double Q, double* E, double* D, double* dQ) {
  if (!(P > 0.0) || !(Q * Q < 6.0)) return false;
  const double e2 = std::exp(2.0 * N), em = std::exp(-N);
  const double pa = std::pow(P, -m.alpha);
  const double pot = m.lam2 / 3.0 * e2 * pa;
  const double mat = m.om * em * std::exp(m.beta * P);
  const double rad = m.orad * em * em;
  const double e = (rad + mat + pot) / (1.0 - Q * Q / 6.0);
  const double d = -Q * Q * e / 3.0 + pot - rad - 0.5 * mat;
  const double force = m.alpha * m.lam2 * e2 * pa / P - 3.0 * m.beta * mat;
  *E = e;
  *D = d;
  *dQ = (force - (2.0 * e + d) * Q) / e;
  return std::isfinite(e) && std::isfinite(*dQ);
}

bool rhs(const Model& m, double N, const double* y, double* f) {
  double E, D, dQ;
  if (!eval(m, N, y[0], y[1], &E, &D, &dQ)) return false;
  f[0] = y[1];
  f[1] = dQ;
  return true;
}

// Dormand-Prince 5(4) tableau
constexpr double c2 = 1.0 / 5, c3 = 3.0 / 10, c4 = 4.0 / 5, c5 = 8.0 / 9;
constexpr double a21 = 1.0 / 5;
constexpr double a31 = 3.0 / 40, a32 = 9.0 / 40;
constexpr double a41 = 44.0 / 45, a42 = -56.0 / 15, a43 = 32.0 / 9;
constexpr double a51 = 19372.0 / 6561, a52 = -25360.0 / 2187, a53 = 64448.0 / 6561,
                 a54 = -212.0 / 729;
constexpr double a61 = 9017.0 / 3168, a62 = -355.0 / 33, a63 = 46732.0 / 5247, a64 = 49.0 / 176,
                 a65 = -5103.0 / 18656;
constexpr double b1 = 35.0 / 384, b3 = 500.0 / 1113, b4 = 125.0 / 192, b5 = -2187.0 / 6784,
                 b6 = 11.0 / 84;
// fifth- minus fourth-order weights (the error estimate)
constexpr double e1 = b1 - 5179.0 / 57600, e3 = b3 - 7571.0 / 16695, e4 = b4 - 393.0 / 640,
                 e5 = b5 + 92097.0 / 339200, e6 = b6 - 187.0 / 2100, e7 = -1.0 / 40;

struct Stepper {
  const Model& m;
  double rtol, atol;
  double h;  // step size carried between calls
  long steps = 0;

  // advance y from N0 to N1 exactly; false if the state leaves the domain
  bool advance(double N0, double N1, double* y) {
    double N = N0;
    double k1[2], k2[2], k3[2], k4[2], k5[2], k6[2], k7[2], yt[2], y5[2];
    if (!rhs(m, N, y, k1)) return false;
    int guard = 0;
    while (N < N1) {
      if (++guard > 1000000) return false;
      double hs = std::fmin(h, N1 - N);
      const bool last = hs >= N1 - N;
      bool ok = true;
      for (int i = 0; i < 2; ++i) yt[i] = y[i] + hs * a21 * k1[i];
      ok = ok && rhs(m, N + c2 * hs, yt, k2);
      for (int i = 0; i < 2 && ok; ++i) yt[i] = y[i] + hs * (a31 * k1[i] + a32 * k2[i]);
      ok = ok && rhs(m, N + c3 * hs, yt, k3);
      for (int i = 0; i < 2 && ok; ++i)
        yt[i] = y[i] + hs * (a41 * k1[i] + a42 * k2[i] + a43 * k3[i]);
      ok = ok && rhs(m, N + c4 * hs, yt, k4);
      for (int i = 0; i < 2 && ok; ++i)
        yt[i] = y[i] + hs * (a51 * k1[i] + a52 * k2[i] + a53 * k3[i] + a54 * k4[i]);
      ok = ok && rhs(m, N + c5 * hs, yt, k5);
      for (int i = 0; i < 2 && ok; ++i)
        yt[i] = y[i] + hs * (a61 * k1[i] + a62 * k2[i] + a63 * k3[i] + a64 * k4[i] + a65 * k5[i]);
      ok = ok && rhs(m, N + hs, yt, k6);
      for (int i = 0; i < 2 && ok; ++i)
        y5[i] = y[i] + hs * (b1 * k1[i] + b3 * k3[i] + b4 * k4[i] + b5 * k5[i] + b6 * k6[i]);
      const double Nn = last ? N1 : N + hs;
      ok = ok && rhs(m, Nn, y5, k7);
      double err = 0.0;
      if (ok) {
        for (int i = 0; i < 2; ++i) {
          const double d = hs * (e1 * k1[i] + e3 * k3[i] + e4 * k4[i] + e5 * k5[i] +
                                 e6 * k6[i] + e7 * k7[i]);
          const double sc = atol + rtol * std::fmax(std::fabs(y[i]), std::fabs(y5[i]));
          err = std::fmax(err, std::fabs(d) / sc);
        }
        ok = std::isfinite(err);
      }
      if (ok && err <= 1.0) {
        N = Nn;
        y[0] = y5[0];
        y[1] = y5[1];
        k1[0] = k7[0];
        k1[1] = k7[1];
        ++steps;
        // keep the step that was asked for when the last one was cut short
        const double grow = err > 0.0 ? 0.9 * std::pow(err, -0.2) : 5.0;
        if (!last || hs == h) h = hs * std::fmin(5.0, std::fmax(0.2, grow));
      } else {
        // a rejected step, or one that left the domain: shrink and retry
        const double shrink = ok ? std::fmax(0.1, 0.9 * std::pow(err, -0.25)) : 0.25;
        h = hs * shrink;
        if (h < 1e-14 * (1.0 + std::fabs(N))) return false;
      }
    }
    return true;
  }
};

double omega_radiation(double h, double t_cmb, double n_eff) {
  // black-body photons at t_cmb plus n_eff massless neutrino species at
  // (4/11)^(1/3) of the photon temperature, 7/8 per species for fermions
  const double kB = 1.380649e-23, hbar = 1.054571817e-34, c = 299792458.0, G = 6.67430e-11;
  const double mpc = 3.0856775814913673e22;
  const double kt = kB * t_cmb;
  const double rho_g = kPi * kPi / 15.0 * kt * kt * kt * kt / std::pow(hbar * c, 3) / (c * c);
  const double H0 = 100.0 * h * 1e3 / mpc;
  const double rho_c = 3.0 * H0 * H0 / (8.0 * kPi * G);
  return rho_g / rho_c * (1.0 + n_eff * 7.0 / 8.0 * std::pow(4.0 / 11.0, 4.0 / 3.0));
}

// integrate from N0 to 0 with lambda; H(a=1)/H0 in *h1; optional table rows
// at n_table nodes uniform in N
bool shoot(const Model& m, double N0, double P0, double Q0, double rtol, int n_table,
           double* table, double* h1, long* steps) {
  Stepper st{m, rtol, 1e-20, 1e-3};
  double y[2] = {P0, Q0};
  const int nodes = n_table > 1 ? n_table : 2;
  double Nprev = N0;
  for (int r = 0; r < nodes; ++r) {
    const double N = r == nodes - 1 ? 0.0 : N0 * (1.0 - double(r) / (nodes - 1));
    if (r > 0 && !st.advance(Nprev, N, y)) return false;
    Nprev = N;
    if (table) {
      double E, D, dQ;
      if (!eval(m, N, y[0], y[1], &E, &D, &dQ)) return false;
      const double a = std::exp(N);
      const double hh = std::sqrt(E) / a;
      double* row = table + 6 * (size_t)r;
      row[0] = r == nodes - 1 ? 1.0 : a;
      row[1] = hh;
      row[2] = (D - E) / (a * a);
      row[3] = y[0];
      row[4] = y[1] / a;
      row[5] = hh * y[1];
    }
  }
  double E, D, dQ;
  if (!eval(m, 0.0, y[0], y[1], &E, &D, &dQ)) return false;
  *h1 = std::sqrt(E);
  *steps += st.steps;
  return true;
}

}  // namespace

extern "C" {

int mg_cq_background(const mg_cq_background_params* p, int n_table, double* table,
                     mg_cq_background_info* info) {
  if (!p || !table || n_table < 2) return MG_EINVAL;
  if (!(p->omega_m > 0.0 && p->omega_m < 1.0) || !(p->h > 0.0) || !(p->t_cmb >= 0.0) ||
      !(p->n_eff >= 0.0) || !(p->alpha >= 0.0) || !std::isfinite(p->beta) || !(p->z_init > 0.0) ||
      !(p->phi_init > 0.0) || !std::isfinite(p->dphi_init) || !(p->tol > 0.0))
    return MG_EINVAL;
  Model m{p->omega_m, omega_radiation(p->h, p->t_cmb, p->n_eff), p->alpha, p->beta, 0.0};
  if (!(m.om + m.orad < 1.0)) return MG_EINVAL;
  const double N0 = -std::log1p(p->z_init);
  const double rtol = 1e-12;
  long steps = 0;
  int shots = 0;
  auto g = [&](double lam, double* out) {
    m.lam2 = lam * lam;
    ++shots;
    double h1;
    if (!shoot(m, N0, p->phi_init, p->dphi_init, rtol, 0, nullptr, &h1, &steps)) return false;
    *out = h1 - 1.0;
    return true;
  };
  // bracket: H(a=1) grows with lambda; start from lambda = 1 as the paper does
  double lo = 0.0, hi = 1.0, glo, ghi;
  if (!g(lo, &glo) || !g(hi, &ghi)) return MG_ENAN;
  if (glo > 0.0) return MG_ENOCONV;  // matter and radiation alone already exceed H0
  for (int k = 0; ghi < 0.0; ++k) {
    if (k > 60) return MG_ENOCONV;
    lo = hi;
    glo = ghi;
    hi *= 2.0;
    if (!g(hi, &ghi)) return MG_ENAN;
  }
  // Illinois false position on H(1)/H0 - 1
  double lam = hi;
  int side = 0;
  for (int it = 0; it < 200; ++it) {
    lam = (lo * ghi - hi * glo) / (ghi - glo);
    if (!(lam > lo && lam < hi)) lam = 0.5 * (lo + hi);
    double gm;
    if (!g(lam, &gm)) return MG_ENAN;
    if (std::fabs(gm) <= p->tol || hi - lo <= 4e-16 * hi) break;
    if ((gm > 0.0) == (ghi > 0.0)) {
      hi = lam;
      ghi = gm;
      if (side == -1) glo *= 0.5;
      side = -1;
    } else {
      lo = lam;
      glo = gm;
      if (side == 1) ghi *= 0.5;
      side = 1;
    }
    if (it == 199) return MG_ENOCONV;
  }
  m.lam2 = lam * lam;
  double h1;
  if (!shoot(m, N0, p->phi_init, p->dphi_init, rtol, n_table, table, &h1, &steps)) return MG_ENAN;
  if (info) {
    info->lambda = lam;
    info->omega_r = m.orad;
    info->h_today = h1;
    info->shots = shots;
    info->steps = steps;
  }
  return MG_OK;
}

int mg_cq_background_at(const double* table, int n_table, double a, double* row) {
  if (!table || !row || n_table < 2) return MG_EINVAL;
  const double a0 = table[0], a1 = table[6 * (size_t)(n_table - 1)];
  if (!(a >= a0 && a <= a1)) return MG_EINVAL;
  int lo = 0, hi = n_table - 1;  // table[lo].a <= a <= table[hi].a
  while (hi - lo > 1) {
    const int mid = (lo + hi) / 2;
    if (table[6 * (size_t)mid] <= a) lo = mid;
    else hi = mid;
  }
  const double* r0 = table + 6 * (size_t)lo;
  const double* r1 = table + 6 * (size_t)hi;
  const double t = r1[0] > r0[0] ? (a - r0[0]) / (r1[0] - r0[0]) : 0.0;
  for (int c = 0; c < 6; ++c) row[c] = r0[c] + t * (r1[c] - r0[c]);
  row[0] = a;
  return MG_OK;
}

}  // extern "C"
