// Von Neumann stability scan of the fine and coarse propagators (host only).
//
// On the periodic grid every Fourier mode exp(i(theta_x i + theta_z j)) is
// an invariant subspace of both propagators; on it a step acts as a 3 x 3
// complex matrix (the amplification matrix).  Fine: one three-stage RK-3
// step of the semi-discrete operator with symbol A(theta) is
// I + Z + Z^2/2 + Z^3/6 with Z = dt_f A (the stability polynomial of every
// three-stage third-order Runge-Kutta method on a linear problem).
// Coarse: the product of N_sound forward-backward substep matrices with the
// slow tendency frozen at the start of the step (Section 3.2).  The spectral
// radius is taken from the eigenvalues found by a shifted complex QR
// iteration, which stays accurate at repeated eigenvalues such as the
// identity at theta = 0.
#include <algorithm>
#include <cmath>
#include <complex>
#include <string>

#include "../../include/libpararealhip.h"

typedef std::complex<double> cd;

int pr_validate(const pr_grid* g, double c_s, double U, double dt_f,
                double dt_g, int32_t P, const pr_opts* o, int* nf, int* ng,
                std::string* msg);

namespace {

struct M3 {
  cd a[3][3];
};

M3 mul(const M3& x, const M3& y) {
  M3 r;
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      cd s = 0;
      for (int k = 0; k < 3; ++k) s += x.a[i][k] * y.a[k][j];
      r.a[i][j] = s;
    }
  return r;
}

// Rotation G = [[c, s], [-conj(s), c]] with G [a; b] = [r; 0].
void givens(cd a, cd b, double* c, cd* s) {
  const double aa = std::abs(a), bb = std::abs(b);
  if (bb == 0.0) {
    *c = 1.0;
    *s = 0.0;
    return;
  }
  if (aa == 0.0) {
    *c = 0.0;
    *s = std::conj(b) / bb;
    return;
  }
  const double r = std::hypot(aa, bb);
  *c = aa / r;
  *s = (a / aa) * std::conj(b) / r;
}

double spectral_radius(M3 H) {
  const int n = 3;
  // Hessenberg form: eliminate H[2][0] with a rotation on rows/cols 1, 2.
  {
    double c;
    cd s;
    givens(H.a[1][0], H.a[2][0], &c, &s);
    for (int j = 0; j < n; ++j) {
      const cd x = H.a[1][j], y = H.a[2][j];
      H.a[1][j] = c * x + s * y;
      H.a[2][j] = -std::conj(s) * x + c * y;
    }
    for (int i = 0; i < n; ++i) {
      const cd x = H.a[i][1], y = H.a[i][2];
      H.a[i][1] = c * x + std::conj(s) * y;
      H.a[i][2] = -s * x + c * y;
    }
    H.a[2][0] = 0.0;
  }
  const double eps = 1e-17;
  int hi = n - 1;
  for (int iter = 0; iter < 500 && hi > 0; ++iter) {
    // deflation
    if (std::abs(H.a[hi][hi - 1]) <=
        eps * (std::abs(H.a[hi][hi]) + std::abs(H.a[hi - 1][hi - 1])) + 1e-300) {
      H.a[hi][hi - 1] = 0.0;
      --hi;
      continue;
    }
    int lo = hi - 1;
    while (lo > 0 &&
           std::abs(H.a[lo][lo - 1]) >
               eps * (std::abs(H.a[lo][lo]) + std::abs(H.a[lo - 1][lo - 1])))
      --lo;
    if (lo > 0) H.a[lo][lo - 1] = 0.0;
    // Wilkinson shift from the trailing 2 x 2 block; an exceptional shift
    // every 20 iterations.
    const cd a = H.a[hi - 1][hi - 1], b = H.a[hi - 1][hi], c2 = H.a[hi][hi - 1],
             dd = H.a[hi][hi];
    const cd half = 0.5 * (a - dd);
    const cd disc = std::sqrt(half * half + b * c2);
    const cd l1 = 0.5 * (a + dd) + disc, l2 = 0.5 * (a + dd) - disc;
    cd mu = std::abs(l1 - dd) < std::abs(l2 - dd) ? l1 : l2;
    if (iter % 20 == 19) mu += 0.75 * std::abs(H.a[hi][hi - 1]);
    double cs[3];
    cd sn[3];
    for (int k = lo; k <= hi; ++k) H.a[k][k] -= mu;
    for (int k = lo; k < hi; ++k) {
      givens(H.a[k][k], H.a[k + 1][k], &cs[k], &sn[k]);
      for (int j = k; j < n; ++j) {
        const cd x = H.a[k][j], y = H.a[k + 1][j];
        H.a[k][j] = cs[k] * x + sn[k] * y;
        H.a[k + 1][j] = -std::conj(sn[k]) * x + cs[k] * y;
      }
    }
    for (int k = lo; k < hi; ++k) {
      const int top = std::min(k + 2, hi);
      for (int i = 0; i <= top; ++i) {
        const cd x = H.a[i][k], y = H.a[i][k + 1];
        H.a[i][k] = cs[k] * x + std::conj(sn[k]) * y;
        H.a[i][k + 1] = -sn[k] * x + cs[k] * y;
      }
    }
    for (int k = lo; k <= hi; ++k) H.a[k][k] += mu;
  }
  double r = 0.0;
  for (int k = 0; k < n; ++k) r = std::max(r, std::abs(H.a[k][k]));
  return r;
}

// R(Z) = I + Z + Z^2/2 + Z^3/6 of Z = dt A.
M3 rk3_amplification(M3 Z, double dt) {
  for (auto& row : Z.a)
    for (auto& v : row) v *= dt;
  const M3 Z2 = mul(Z, Z), Z3 = mul(Z2, Z);
  M3 R;
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j)
      R.a[i][j] = (i == j ? 1.0 : 0.0) + Z.a[i][j] + 0.5 * Z2.a[i][j] +
                  Z3.a[i][j] / 6.0;
  return R;
}

// Symbol matrix of the Section 3.1 right-hand side: scalar advection
// symbol adv on the diagonal, centred second-order acoustics.
M3 acoustic2(cd adv, cd dx2, cd dz2, double c_s) {
  M3 Z;
  Z.a[0][0] = adv;
  Z.a[0][1] = 0.0;
  Z.a[0][2] = -c_s * dx2;
  Z.a[1][0] = 0.0;
  Z.a[1][1] = adv;
  Z.a[1][2] = -c_s * dz2;
  Z.a[2][0] = -c_s * dx2;
  Z.a[2][1] = -c_s * dz2;
  Z.a[2][2] = adv;
  return Z;
}

}  // namespace

namespace {

// Scan for the pair of the instability example (Section 3.1): F and G are
// both RK-3, with the sixth-order centred and the first-order upwind
// advective symbols along x (U) and z (V).
void scan_rk3(int nx, int nz, double dx, double dz, double c_s, double U,
              double V, double dt_f, double dt_g, int kxn, int kzn,
              double* rho_f, double* rho_g) {
  const cd I(0.0, 1.0);
  const double two_pi = 2.0 * M_PI;
  auto c6 = [&](double t, double h) {
    return I * (45.0 * std::sin(t) - 9.0 * std::sin(2.0 * t) +
                std::sin(3.0 * t)) / (30.0 * h);
  };
  auto up1 = [&](double t, double h, double vel) {
    return vel >= 0 ? (1.0 - std::exp(-I * t)) / h : (std::exp(I * t) - 1.0) / h;
  };
  double rf = 0.0, rg = 0.0;
  for (int a = 0; a < kxn; ++a) {
    const long long kx = kxn == nx ? a : (long long)a * nx / 256;
    const double tx = two_pi * (double)kx / nx;
    for (int b = 0; b < kzn; ++b) {
      const long long kz = kzn == nz ? b : (long long)b * nz / 256;
      const double tz = two_pi * (double)kz / nz;
      const cd dx2 = I * std::sin(tx) / dx, dz2 = I * std::sin(tz) / dz;
      const cd af = -U * c6(tx, dx) - V * c6(tz, dz);
      const cd ag = -U * up1(tx, dx, U) - V * up1(tz, dz, V);
      rf = std::max(rf, spectral_radius(
                            rk3_amplification(acoustic2(af, dx2, dz2, c_s), dt_f)));
      rg = std::max(rg, spectral_radius(
                            rk3_amplification(acoustic2(ag, dx2, dz2, c_s), dt_g)));
    }
  }
  *rho_f = rf;
  *rho_g = rg;
}

}  // namespace

namespace {

// Fifth-order upwind derivative symbol (point weights /(60 h) at offsets
// -3..2 for vel >= 0, mirrored for vel < 0) times -vel.
cd adv5_symbol(double t, double h, double vel) {
  static const double wpos[6] = {-2.0, 15.0, -60.0, 20.0, 30.0, -3.0};
  static const double wneg[6] = {3.0, -30.0, -20.0, 60.0, -15.0, 2.0};
  const double* w = vel >= 0 ? wpos : wneg;
  const int m0 = vel >= 0 ? -3 : -2;
  const cd I(0.0, 1.0);
  cd a = 0.0;
  for (int k = 0; k < 6; ++k) a += w[k] * std::exp(I * (double)(m0 + k) * t);
  return -vel * a / (60.0 * h);
}

// First-order (or, with order 3, third-order) upwind derivative symbol
// times -vel; third order has point weights (1, -6, 3, 2)/6 at offsets
// -2..1 for vel >= 0, mirrored for vel < 0.
cd adv1_symbol(double t, double h, double vel, int order = 1) {
  const cd I(0.0, 1.0);
  if (order == 3) {
    auto e = [&](int m) { return std::exp(I * (double)m * t); };
    const cd a = vel >= 0 ? e(-2) - 6.0 * e(-1) + 3.0 + 2.0 * e(1)
                          : -2.0 * e(-1) - 3.0 + 6.0 * e(1) - e(2);
    return -vel * a / (6.0 * h);
  }
  return vel >= 0 ? -vel * (1.0 - std::exp(-I * t)) / h
                  : -vel * (std::exp(I * t) - 1.0) / h;
}

// Scan of the Section 3.2 pair for the constant velocity (U, V): F is RK-3
// of fifth-order upwind advection, centred acoustics of the fine order and
// grad-div damping; G is N_sound forward-backward substeps with the frozen
// upwind slow tendency of the coarse order.
void scan_split(int nx, int nz, double dx, double dz, double c_s, double U,
                double V, double dt_f, double dt_g, const pr_opts* o,
                int kxn, int kzn, double* rho_f, double* rho_g) {
  const double ax_f = o->nu_f * dx * dx / dt_f, az_f = o->nu_f * dz * dz / dt_f;
  const double dtau = dt_g / o->n_sound;
  const double ax_c = o->nu_c * dx * dx / dtau, az_c = o->nu_c * dz * dz / dtau;
  const bool fourth = o->fine_acoustic_order != 2;
  const double two_pi = 2.0 * M_PI;
  const cd I(0.0, 1.0);
  double rf = 0.0, rg = 0.0;
  for (int a = 0; a < kxn; ++a) {
    const long long kx = kxn == nx ? a : (long long)a * nx / 256;
    const double tx = two_pi * (double)kx / nx;
    for (int b = 0; b < kzn; ++b) {
      const long long kz = kzn == nz ? b : (long long)b * nz / 256;
      const double tz = two_pi * (double)kz / nz;
      const cd a5 = adv5_symbol(tx, dx, U) + adv5_symbol(tz, dz, V);
      const cd dx2 = I * std::sin(tx) / dx, dz2 = I * std::sin(tz) / dz;
      const cd dxf = fourth ? I * (8.0 * std::sin(tx) - std::sin(2.0 * tx)) / (6.0 * dx) : dx2;
      const cd dzf = fourth ? I * (8.0 * std::sin(tz) - std::sin(2.0 * tz)) / (6.0 * dz) : dz2;
      const double gxx = -4.0 * std::pow(std::sin(0.5 * tx), 2) / (dx * dx);
      const double gzz = -4.0 * std::pow(std::sin(0.5 * tz), 2) / (dz * dz);
      const double gxz = -std::sin(tx) * std::sin(tz) / (dx * dz);
      M3 Z;
      Z.a[0][0] = a5 + ax_f * gxx;
      Z.a[0][1] = ax_f * gxz;
      Z.a[0][2] = -c_s * dxf;
      Z.a[1][0] = az_f * gxz;
      Z.a[1][1] = a5 + az_f * gzz;
      Z.a[1][2] = -c_s * dzf;
      Z.a[2][0] = -c_s * dxf;
      Z.a[2][1] = -c_s * dzf;
      Z.a[2][2] = a5;
      rf = std::max(rf, spectral_radius(rk3_amplification(Z, dt_f)));
      // coarse step
      const cd a1 = adv1_symbol(tx, dx, U, o->coarse_order) +
                    adv1_symbol(tz, dz, V, o->coarse_order);
      M3 Y;
      for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) Y.a[i][j] = i == j ? 1.0 : 0.0;
      for (int s = 0; s < o->n_sound; ++s) {
        cd un[3], wn[3], pn[3];
        for (int j = 0; j < 3; ++j) {
          const cd u = Y.a[0][j], wv = Y.a[1][j], p = Y.a[2][j];
          un[j] = u + dtau * ((j == 0 ? a1 : 0.0) - c_s * dx2 * p +
                              ax_c * (gxx * u + gxz * wv));
          wn[j] = wv + dtau * ((j == 1 ? a1 : 0.0) - c_s * dz2 * p +
                               az_c * (gzz * wv + gxz * u));
        }
        for (int j = 0; j < 3; ++j)
          pn[j] = Y.a[2][j] +
                  dtau * ((j == 2 ? a1 : 0.0) - c_s * (dx2 * un[j] + dz2 * wn[j]));
        for (int j = 0; j < 3; ++j) {
          Y.a[0][j] = un[j];
          Y.a[1][j] = wn[j];
          Y.a[2][j] = pn[j];
        }
      }
      rg = std::max(rg, spectral_radius(Y));
    }
  }
  *rho_f = rf;
  *rho_g = rg;
}

}  // namespace

int pr_check_stability_impl(const pr_grid* g, double c_s, double U,
                            double dt_f, double dt_g, const pr_opts* o,
                            double* rho_f, double* rho_g) {
  const int nx = g->nx, nz = g->nz;
  const bool all = (long long)nx * nz <= 65536;
  const int kxn = all || nx <= 256 ? nx : 256;
  const int kzn = all || nz <= 256 ? nz : 256;
  const double dx = g->Lx / nx, dz = g->Lz / nz;
  if (o->scheme == PR_SCHEME_RK3) {
    scan_rk3(nx, nz, dx, dz, c_s, U, o->V, dt_f, dt_g, kxn, kzn, rho_f, rho_g);
    return PR_OK;
  }
  if (o->gamma == 0.0) {
    scan_split(nx, nz, dx, dz, c_s, U, o->V, dt_f, dt_g, o, kxn, kzn, rho_f,
               rho_g);
    return PR_OK;
  }
  // Frozen coefficients at the extreme velocities of the rows (x) and of
  // the columns (z): U + gamma (z_j - Lz/2) and V - gamma (x_i - Lx/2).
  const double zlo = 0.5 * dz - 0.5 * g->Lz, zhi = (nz - 0.5) * dz - 0.5 * g->Lz;
  const double xlo = 0.5 * dx - 0.5 * g->Lx, xhi = (nx - 0.5) * dx - 0.5 * g->Lx;
  const double us[2] = {U + o->gamma * zlo, U + o->gamma * zhi};
  const double vs[2] = {o->V - o->gamma * xlo, o->V - o->gamma * xhi};
  double rf = 0.0, rg = 0.0;
  for (double u : us)
    for (double v : vs) {
      double f, gg;
      scan_split(nx, nz, dx, dz, c_s, u, v, dt_f, dt_g, o, kxn, kzn, &f, &gg);
      rf = std::max(rf, f);
      rg = std::max(rg, gg);
    }
  *rho_f = rf;
  *rho_g = rg;
  return PR_OK;
}

extern "C" int pr_check_stability(const pr_grid* g, double c_s, double U,
                                  double dt_f, double dt_g, const pr_opts* o,
                                  double* rho_f, double* rho_g) {
  pr_opts def;
  pr_opts_default(&def);
  if (!o) o = &def;
  if (!rho_f || !rho_g) return PR_EINVAL;
  int nf, ng;
  // Stability does not depend on P; validate with one slice of length T.
  if (pr_validate(g, c_s, U, dt_f, dt_g, 1, o, &nf, &ng, nullptr) != PR_OK) {
    // Steps need not divide T for the scan itself; check the rest.
    if (!g || g->nx < 8 || g->nz < 8 || !(dt_f > 0) || !(dt_g > 0) ||
        o->n_sound < 1 || !(g->Lx > 0) || !(g->Lz > 0))
      return PR_EINVAL;
  }
  return pr_check_stability_impl(g, c_s, U, dt_f, dt_g, o, rho_f, rho_g);
}
