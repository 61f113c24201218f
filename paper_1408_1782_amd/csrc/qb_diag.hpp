// Diagnostics of a Wigner state, one workgroup per cell, float64
// arithmetic whatever the state's precision:
//   * local entropy S = -h^2 sum_v tr[W log W + W~ log W~], W~ = 1 - W
//     (Sec. 2, eq. entropy_def);
//   * entropy production density sigma = -h^2 sum_v tr[(log W - log W~) C]
//     (the integrand of the H-theorem of Sec. 2), given C = C[W];
//   * quantum relative entropy to a Fermi-Dirac state F,
//     h^2 sum_v tr[W (log W - log F) + W~ (log W~ - log F~)]
//     (Sec. 5, eq. relentropy_hom), for a global state at rest and for the
//     local fit (eq. relentropy_local);
//   * the eigenvalue range of W(v) (Sec. 5);
//   * the local Fermi-Dirac fit: velocity u from the momentum, per-spin
//     densities = eigenvalues of the spin density, temperature from the
//     internal energy through the closed forms of eq. momentsFermiDirac,
//     spin basis = eigenbasis of the spin density (Sec. 5).
// A 2x2 Hermitian W = w0 + w.sigma has eigenvalues w0 +- |w| with
// projectors (1 +- n.sigma)/2, n = w/|w|, so every matrix function is
// f(W) = sum_+- f(lambda_+-) (1 +- n.sigma)/2 and tr[f(W) A] =
// sum_+- f(lambda_+-) (a0 +- n.a).  Eigenvalues are clamped into [0, 1] and
// logarithms read as log(max(x, 1e-300)), so 0 log 0 = 0.
#pragma once
#include <hip/hip_runtime.h>

#include "qb_fft.hpp"  // kPi

namespace qb {

constexpr int kDiagFields = 11;

// Global Fermi-Dirac state at rest: 1/kT, chemical potentials and the Bloch
// vector of the spin-up projector.
struct FdGlobal {
  double inv_kT, mu_up, mu_down, n[3];
  int valid;
};

__device__ __forceinline__ double dlog(double x) { return log(fmax(x, 1e-300)); }
// log(1 + e^x) without overflow
__device__ __forceinline__ double softplus(double x) { return fmax(x, 0.0) + log1p(exp(-fabs(x))); }

// Li_2(y) = sum_k y^k / k^2 for 0 <= y <= 1/2 (terms fall at least as 2^-k)
__device__ inline double li2_series(double y) {
  double s = 0.0, p = y;
  for (int k = 1; k < 80; ++k) {
    const double t = p / ((double)k * k);
    s += t;
    if (t < 1e-18 * s) break;
    p *= y;
  }
  return s;
}

// -Li_2(1 - e^a) for a > 0, i.e. -Li_2(-z) with z = e^a - 1: for
// 1 - e^a >= -1 (a <= log 2) by Landen's identity Li_2(x) =
// -Li_2(x / (x - 1)) - log^2(1 - x) / 2, whose argument x / (x - 1) =
// 1 - e^{-a} lies in (0, 1/2]; below -1 by the inversion formula
// Li_2(x) + Li_2(1/x) = -pi^2/6 - log^2(-x) / 2 and Landen's identity for
// 1/x, whose argument is e^{-a} < 1/2.
__device__ inline double neg_li2_1mexp(double a) {
  const double PI2_6 = 1.6449340668482264365;
  if (a <= 0.69314718055994530942) return li2_series(-expm1(-a)) + 0.5 * a * a;
  const double q = exp(-a), lq = log1p(-q);
  return PI2_6 + 0.5 * (a + lq) * (a + lq) - li2_series(q) - 0.5 * lq * lq;
}

// Internal energy per particle of the Fermi-Dirac state with per-spin
// densities r_s at temperature kT: with a_s = r_s / (2 pi kT) =
// log(1 + e^{mu_s/kT}), eps = kT sum_s (-Li_2(-e^{mu_s/kT})) / sum_s a_s
// (eq. momentsFermiDirac).
__device__ inline double fd_eps(double kT, double r_up, double r_dn) {
  const double a = r_up / (2.0 * kPi * kT), b = r_dn / (2.0 * kPi * kT);
  return kT * (neg_li2_1mexp(a) + neg_li2_1mexp(b)) / (a + b);
}

// Pauli components (Hermitian part) of point e of cell c, API layout
template <typename TA>
__device__ __forceinline__ void api_point(const TA* __restrict__ W, size_t pt, double w[4]) {
  const TA* p = W + pt * 8;
  const double a00 = (double)p[0], r01 = (double)p[2], i01 = (double)p[3], r10 = (double)p[4], i10 = (double)p[5],
               a11 = (double)p[6];
  w[0] = 0.5 * (a00 + a11);
  w[1] = 0.5 * (r01 + r10);
  w[2] = 0.5 * (i10 - i01);
  w[3] = 0.5 * (a00 - a11);
}

// eigenvalues (unclamped) and the unit Bloch vector (e_3 when w = 0)
__device__ __forceinline__ void eig2(const double w[4], double& lp, double& lm, double n[3]) {
  const double r = sqrt(w[1] * w[1] + w[2] * w[2] + w[3] * w[3]);
  lp = w[0] + r;
  lm = w[0] - r;
  if (r > 0.0) {
    n[0] = w[1] / r;
    n[1] = w[2] / r;
    n[2] = w[3] / r;
  } else {
    n[0] = n[1] = 0.0;
    n[2] = 1.0;
  }
}

__device__ __forceinline__ double clamp01(double x) { return fmin(fmax(x, 0.0), 1.0); }

// tr[W log W + W~ log W~] at one point
__device__ __forceinline__ double neg_entropy_density(double lp, double lm) {
  const double a = clamp01(lp), b = clamp01(lm);
  return a * dlog(a) + (1.0 - a) * dlog(1.0 - a) + b * dlog(b) + (1.0 - b) * dlog(1.0 - b);
}

// tr[W log F + W~ log F~] for F = sum_s f_s P_s with spin-up projector
// (1 + m.sigma)/2 and f_s = 1 / (e^{x_s} + 1): log f = -softplus(x),
// log(1 - f) = -softplus(-x)
__device__ __forceinline__ double cross_term(const double w[4], const double m[3], double xu, double xd) {
  const double wm = w[1] * m[0] + w[2] * m[1] + w[3] * m[2];
  const double pu = w[0] + wm, pd = w[0] - wm;  // tr[W P_s]
  return -softplus(xu) * pu - softplus(-xu) * (1.0 - pu) - softplus(xd) * pd - softplus(-xd) * (1.0 - pd);
}

template <int K>
__device__ __forceinline__ void block_sum(double (*red)[256], double (&v)[K]) {
  for (int k = 0; k < K; ++k) red[k][threadIdx.x] = v[k];
  __syncthreads();
  for (int o = blockDim.x / 2; o > 0; o >>= 1) {
    if (threadIdx.x < o)
      for (int k = 0; k < K; ++k) red[k][threadIdx.x] += red[k][threadIdx.x + o];
    __syncthreads();
  }
  for (int k = 0; k < K; ++k) v[k] = red[k][0];
  __syncthreads();
}

// One workgroup of 256 threads per cell.  out[cell][0..10]: entropy,
// entropy production density, relative entropy to the global state,
// relative entropy to the local fit, smallest and largest eigenvalue, kT,
// mu_up, mu_down, u_x, u_y of the fit (NaN fit fields and relative entropy
// where the fit has no solution).
template <typename TA>
__global__ __launch_bounds__(256) void k_diagnostics(const TA* __restrict__ W, const TA* __restrict__ C,
                                                     FdGlobal g, double* __restrict__ out, int N, double L) {
  const int cell = blockIdx.x;
  const int per = N * N;
  const double h = 2.0 * L / N;
  const size_t base = (size_t)cell * per;
  __shared__ double red[12][256];
  __shared__ double mn[256], mx[256];
  __shared__ double fit[9];  // kT, mu_up, mu_down, ux, uy, n (3), valid
  // pass 1: moments, entropy, entropy production, global relative entropy,
  // eigenvalue range
  double acc[10] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
  double lo = 1e300, hi = -1e300;
  for (int e = threadIdx.x; e < per; e += blockDim.x) {
    const double vx = h * (e / N - N / 2), vy = h * (e % N - N / 2);
    double w[4], n[3], lp, lm;
    api_point(W, base + e, w);
    eig2(w, lp, lm, n);
    lo = fmin(lo, lm);
    hi = fmax(hi, lp);
    for (int k = 0; k < 4; ++k) acc[k] += w[k];
    const double tr = 2.0 * w[0];
    acc[4] += vx * tr;
    acc[5] += vy * tr;
    acc[6] += 0.5 * (vx * vx + vy * vy) * tr;
    const double nes = neg_entropy_density(lp, lm);
    acc[7] -= nes;
    if (C) {
      double c[4];
      api_point(C, base + e, c);
      const double a = clamp01(lp), b = clamp01(lm);
      const double gp = dlog(a) - dlog(1.0 - a), gm = dlog(b) - dlog(1.0 - b);
      const double cn = c[1] * n[0] + c[2] * n[1] + c[3] * n[2];
      acc[8] -= gp * (c[0] + cn) + gm * (c[0] - cn);
    }
    if (g.valid) {
      const double om = 0.5 * (vx * vx + vy * vy);
      acc[9] += nes - cross_term(w, g.n, (om - g.mu_up) * g.inv_kT, (om - g.mu_down) * g.inv_kT);
    }
  }
  mn[threadIdx.x] = lo;
  mx[threadIdx.x] = hi;
  block_sum<10>(red, acc);
  for (int o = blockDim.x / 2; o > 0; o >>= 1) {
    if (threadIdx.x < o) {
      mn[threadIdx.x] = fmin(mn[threadIdx.x], mn[threadIdx.x + o]);
      mx[threadIdx.x] = fmax(mx[threadIdx.x], mx[threadIdx.x + o]);
    }
    __syncthreads();
  }
  // local Fermi-Dirac fit (one thread): rho = h^2 sum w, n = tr rho,
  // u = p / n, eps = e / n - |u|^2 / 2; the temperature solves
  // eps_FD(kT) = eps by bisection in log kT over [r_up / (1200 pi), eps]
  // (eps_FD(kT) >= kT for fermions; below that bracket e^{a_s} leaves the
  // float64 range)
  if (threadIdx.x == 0) {
    const double h2 = h * h;
    const double r0 = h2 * acc[0], r1 = h2 * acc[1], r2 = h2 * acc[2], r3 = h2 * acc[3];
    const double dens = 2.0 * r0;
    const double ux = h2 * acc[4] / dens, uy = h2 * acc[5] / dens;
    const double eps = h2 * acc[6] / dens - 0.5 * (ux * ux + uy * uy);
    const double rv = sqrt(r1 * r1 + r2 * r2 + r3 * r3);
    const double ru = r0 + rv, rd = r0 - rv;
    double kT = NAN, mu = NAN, md = NAN;
    bool ok = rd > 0.0 && eps > 0.0;
    double a = ok ? log(ru / (1200.0 * kPi)) : 0.0, b = ok ? log(eps) : 0.0;
    ok = ok && a < b && fd_eps(exp(a), ru, rd) - eps < 0.0;
    if (ok) {
      if (fd_eps(exp(b), ru, rd) - eps <= 0.0) {
        a = b;
      } else {
        for (int it = 0; it < 200 && b - a > 1e-15 * fmax(1.0, fabs(a)); ++it) {
          const double c = 0.5 * (a + b);
          if (fd_eps(exp(c), ru, rd) - eps < 0.0)
            a = c;
          else
            b = c;
        }
        a = 0.5 * (a + b);
      }
      kT = exp(a);
      const double au = ru / (2.0 * kPi * kT), ad = rd / (2.0 * kPi * kT);
      mu = kT * (au + log1p(-exp(-au)));  // kT log(e^{a} - 1)
      md = kT * (ad + log1p(-exp(-ad)));
    }
    fit[0] = kT;
    fit[1] = mu;
    fit[2] = md;
    fit[3] = ux;
    fit[4] = uy;
    fit[5] = rv > 0.0 ? r1 / rv : 0.0;
    fit[6] = rv > 0.0 ? r2 / rv : 0.0;
    fit[7] = rv > 0.0 ? r3 / rv : 1.0;
    fit[8] = ok ? 1.0 : 0.0;
  }
  __syncthreads();
  // pass 2: relative entropy to the local fit W_FD(v - u)
  double loc[1] = {0.0};
  const bool ok = fit[8] != 0.0;
  if (ok) {
    const double ikT = 1.0 / fit[0];
    const double m[3] = {fit[5], fit[6], fit[7]};
    for (int e = threadIdx.x; e < per; e += blockDim.x) {
      const double vx = h * (e / N - N / 2) - fit[3], vy = h * (e % N - N / 2) - fit[4];
      const double om = 0.5 * (vx * vx + vy * vy);
      double w[4], n[3], lp, lm;
      api_point(W, base + e, w);
      eig2(w, lp, lm, n);
      loc[0] += neg_entropy_density(lp, lm) - cross_term(w, m, (om - fit[1]) * ikT, (om - fit[2]) * ikT);
    }
  }
  block_sum<1>(red, loc);
  if (threadIdx.x == 0) {
    const double h2 = h * h;
    double* o = out + (size_t)cell * kDiagFields;
    o[0] = h2 * acc[7];
    o[1] = h2 * acc[8];
    o[2] = h2 * acc[9];
    o[3] = ok ? h2 * loc[0] : NAN;
    o[4] = mn[0];
    o[5] = mx[0];
    for (int k = 0; k < 5; ++k) o[6 + k] = fit[k];
  }
}

}  // namespace qb
