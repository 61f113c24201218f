// Reverse-mode kernels: vector-Jacobian products of the collision operator
// (Sec. 3.2), the limited transport step (eq. slopeLimiterStep with
// eq. minmod, Sec. 2 walls) and the Heun stages with the field term.
//
// Conventions.  Real fields carry ordinary gradients (dl = sum g dx).  A
// complex array that is a linear image of real data carries a "bilinear"
// cotangent lam with dl = Re sum lam dx.  The unnormalized 2D DFT matrix F
// (e^{-}) and its conjugate (e^{+}) are symmetric, so under this pairing
//   fwd2 (F, row real -> col spec) transposes to F from col spec to row:
//        F c = conj(inv2(conj c));
//   inv2 (conj F, col spec -> row real) transposes to conj F from row to
//        col spec: conj(F) r = conj(fwd2(conj r));
// a pointwise product transposes to the same product, and taking a real
// part transposes to embedding a real cotangent.  Every cotangent of a
// spectrum built here is Hermitian, so two of them pack into one complex
// array exactly as two real fields do.
#pragma once
#include "qb_kernels.hpp"

namespace qb {

// ------------------------------------------------------------------ layout
// API cotangent G (torch convention dl = Re sum conj(G) dW) of a state
// W = sum_mu w_mu sigma_mu -> Pauli gradient g_mu = Re tr(sigma_mu G).
template <typename T, typename TA>
__global__ void k_api_to_cot(const TA* __restrict__ G, T* __restrict__ g, int ncells, int N, int Nx) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  const int per = N * N;
  if (idx >= ncells * per) return;
  const TA* m = G + (size_t)idx * 8;  // G00 G01 G10 G11, each (re, im)
  const double g00r = m[0], g01r = m[2], g01i = m[3], g10r = m[4], g10i = m[5], g11r = m[6];
  const size_t cs = (size_t)Nx * per;
  g[idx] = (T)(g00r + g11r);
  g[cs + idx] = (T)(g10r + g01r);
  g[2 * cs + idx] = (T)(g10i - g01i);
  g[3 * cs + idx] = (T)(g00r - g11r);
}

// Pauli gradient g of w_mu = (1/2) Re tr(sigma_mu W) -> API cotangent
// G = (1/2) sum_mu g_mu sigma_mu.
template <typename T, typename TA>
__global__ void k_cot_to_api(const T* __restrict__ g, TA* __restrict__ G, int ncells, int N, int Nx) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  const int per = N * N;
  if (idx >= ncells * per) return;
  const size_t cs = (size_t)Nx * per;
  const T a0 = (T)0.5 * g[idx], a1 = (T)0.5 * g[cs + idx], a2 = (T)0.5 * g[2 * cs + idx],
          a3 = (T)0.5 * g[3 * cs + idx];
  TA* m = G + (size_t)idx * 8;
  m[0] = (TA)(a0 + a3);
  m[1] = (TA)0;
  m[2] = (TA)a1;
  m[3] = (TA)(-a2);
  m[4] = (TA)a1;
  m[5] = (TA)a2;
  m[6] = (TA)(a0 - a3);
  m[7] = (TA)0;
}

// ------------------------------------------------------------------ output stage
// Transpose of k_combine: the map r -> c is E . Proj with Proj the real,
// symmetric band projection inv2 . (mask / P^2) . fwd2 and E the restriction
// to the even points, so the cotangent of the assembled fields is
// Proj(E^T lam): lam placed on the even points, projected onto Xi.  Its
// spectrum (packed pairs (0 + i1), (2 + i3), col spec) goes to lamh.
template <typename T, int P, int E>
__global__ __launch_bounds__((Fft2<T, P, E>::NT)) void k_lam_in(DevPlan<T> d, const T* __restrict__ lam,
                                                                int cell0) {
  using K = Kern<T, P, E>;
  constexpr unsigned S = sizeof(T);
  __shared__ T smem[K::LDS];
  Fft2<T, P, E> eng;
  setup(eng, smem, d.tw);
  const int lc = blockIdx.x;
  const int cell = cell0 + lc;
  const int N = P / 2;
  const unsigned vo = threadIdx.x * S;
  const size_t cs = (size_t)d.Nx * N * N;
  const rsrc_t ro = mkbuf(d.lamP + (size_t)lc * 4 * K::FSZ, 4 * K::FSZ);
  const rsrc_t rh = mkbuf(d.lamh + (size_t)lc * 4 * K::FSZ, 4 * K::FSZ);
  const int y = eng.line;
  const bool on_grid = ((eng.q | y) & 1) == 0;
  const int bx = centered<P>(eng.line);
  const bool kx_in = bx > -N / 2 && bx < N / 2;
  const T sc = (T)1 / (T)(P * P);
#pragma unroll 1
  for (int pr = 0; pr < 2; ++pr) {
    T zr[E], zi[E];
    const T* la = lam + (2 * pr) * cs + (size_t)cell * N * N + (centered<P>(y) / 2 + N / 2);
    const T* lb = la + cs;
#pragma unroll
    for (int n = 0; n < E; ++n) {
      const int i = vel_index<P, K::TPR>(eng.q, n);
      zr[n] = on_grid ? la[i * N] : (T)0;
      zi[n] = on_grid ? lb[i * N] : (T)0;
    }
    eng.fwd2(zr, zi);
#pragma unroll
    for (int k = 0; k < E; ++k) {
      const int by = centered<P>(eng.bk(k));
      const bool in = kx_in && by > -N / 2 && by < N / 2;
      zr[k] = in ? zr[k] * sc : (T)0;
      zi[k] = in ? zi[k] * sc : (T)0;
      // spectrum of the projected cotangent (packed pair), kept for k_i3_vjp
      bst<T>(rh, zr[k], vo, ((2 * pr) * K::FSZ + k * K::NT) * S);
      bst<T>(rh, zi[k], vo, ((2 * pr + 1) * K::FSZ + k * K::NT) * S);
    }
    eng.inv2(zr, zi);
#pragma unroll
    for (int n = 0; n < E; ++n) {
      bst<T>(ro, zr[n], vo, ((2 * pr) * K::FSZ + n * K::NT) * S);
      bst<T>(ro, zi[n], vo, ((2 * pr + 1) * K::FSZ + n * K::NT) * S);
    }
  }
}

// Transpose of k_assemble (pointwise on the P grid).  From the cotangent
// lam of the assembled fields r_mu:
//   acot[0..2]  cotangent of the I_1 fields g_l
//   acot[3..6]  cotangent of the I_4 fields y_mu
//   acot[7]     cotangent of the I_2 accumulator S
//   acot[8..11] cotangent of the I_3 sums b_nu
//   acot[12..15] the explicit dependence of r on w_mu
// Part 0 writes acot[0..11], which need only lam and w; part 1 writes
// acot[12..15] from the forward fields g, y (terms[0..6]) and S (the sum
// of its per-component parts terms[7..10]), which k_terms_vjp produces.
template <typename T>
__global__ void k_assemble_vjp(DevPlan<T> d, int ncells, int fsz, int part) {
  const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (size_t)ncells * fsz) return;
  const size_t cell = idx / fsz, e = idx % fsz;
  const T* lp = d.lamP + cell * 4 * fsz + e;
  const T* wp = d.wP + cell * 5 * fsz + e;
  const T l0 = lp[0], l1 = lp[fsz], l2 = lp[2 * fsz], l3 = lp[3 * fsz];
  const T w0 = wp[0], w1 = wp[fsz], w2 = wp[2 * fsz], w3 = wp[3 * fsz];
  const T pi = (T)kPi, two = (T)2, tp = (T)(2.0 * kPi);
  T* o = d.acot + cell * 16 * fsz + e;
  if (part == 0) {
    // r_k = -2 (g x w)_k + ...  (C_c);  r_0, r_k of A, B, Cq (see k_assemble)
    o[0] = two * (w3 * l2 - w2 * l3);
    o[fsz] = two * (w1 * l3 - w3 * l1);
    o[2 * fsz] = two * (w2 * l1 - w1 * l2);
    o[3 * fsz] = tp * (w0 * l0 + w1 * l1 + w2 * l2 + w3 * l3);
    o[4 * fsz] = tp * (-w1 * l0 - w0 * l1);
    o[5 * fsz] = tp * (-w2 * l0 - w0 * l2);
    o[6 * fsz] = tp * (-w3 * l0 - w0 * l3);
    o[7 * fsz] = pi * (two * ((T)1 - w0) * l0 - two * (w1 * l1 + w2 * l2 + w3 * l3));
    o[8 * fsz] = -tp * l0;
    o[9 * fsz] = tp * l1;
    o[10 * fsz] = tp * l2;
    o[11 * fsz] = tp * l3;
    return;
  }
  const T* tr = d.terms + cell * kTermPlanes * fsz + e;
  const T g1 = tr[0], g2 = tr[fsz], g3 = tr[2 * fsz];
  const T y0 = tr[3 * fsz], y1 = tr[4 * fsz], y2 = tr[5 * fsz], y3 = tr[6 * fsz];
  const T Sv = (tr[7 * fsz] + tr[8 * fsz]) + (tr[9 * fsz] + tr[10 * fsz]);
  const T q = pi * (-two * Sv + two * y0);
  o[12 * fsz] = q * l0 - tp * (y1 * l1 + y2 * l2 + y3 * l3);
  o[13 * fsz] = -tp * y1 * l0 + q * l1 - two * g3 * l2 + two * g2 * l3;
  o[14 * fsz] = -tp * y2 * l0 + two * g3 * l1 + q * l2 - two * g1 * l3;
  o[15 * fsz] = -tp * y3 * l0 - two * g2 * l1 + two * g1 * l2 + q * l3;
}

// ------------------------------------------------------------------ I_1, I_4, I_2
// Transpose of k_terms, one workgroup per (cell, task), fused with the
// forward fields the transpose of the assembly needs (k_terms computes
// the same fields; running both here shares their inner transforms).
// Tasks 0..6 (I_1 with l = task + 1, I_4 with g = task - 3), per direction j:
//   forward  a_j = inv2(in_j w_hat_g), c_j = fwd2(f0 a_j), field = Re inv2(sum_j out_j c_j)
//   reverse  b_j = F(out_j d) with d = conj(F) field_bar;
//            f0_bar += Re(a_j b_j);  w_hat_g_bar += in_j conj(F)(f0 b_j)
// The tables in_j, out_j are real and have one parity in k (odd for I_1,
// even for I_4), and w_hat_g, field_bar are spectra of real fields, so
// a_j, b_j are real up to a fixed phase.  Two directions j, j+1 therefore
// share every transform (dir_pair gives the complex coefficients): one
// transform yields a_j + i a_j+1 (up to the phase), one the pair's forward
// contribution, one b_j + i b_j+1, and one the pair's cotangent H, whose
// Hermitian part (H(k) + conj H(-k)) / 2 is the cotangent of w_hat_g;
// k_grad_pre takes that part.
// Tasks 7..10 (I_2, one Pauli component mu = task - 7 each):
//            S = sum_j sum_mu e_mu A_j,mu B_j,mu with A + iB = inv2(w_hat_mu (psi_j + i psi'_j)):
//            w_hat_mu_bar += psi_j conj(F)(S_bar e_mu B) + psi'_j conj(F)(S_bar e_mu A)
//   The two real products go through one transform Z = fwd2(S_bar e_mu (B + iA));
//   (psi_j + i psi'_j) conj(Z) has the cotangent as its Hermitian part.
//   (the component's share sum_j e_mu A B of S goes to terms[task])
// The field cotangents (acot[0..7]) depend only on lam and w, so they are
// ready before this kernel; the dependence of the assembly on the fields
// themselves (acot[12..15]) is formed after it.
// Workgroups of 512 threads or more are held to 128 registers per lane,
// so two of them share a compute unit: the kernel waits on its private
// accumulators between transforms, and a second workgroup fills those
// waits (measured at N = 32 in float64: -11 % with 15 registers spilled).
constexpr int kTermsVjpTasks = kTermPlanes;
template <typename T, int P, int E>
__global__ __launch_bounds__((Fft2<T, P, E>::NT))
__attribute__((amdgpu_waves_per_eu(Fft2<T, P, E>::NT >= 512 ? 4 : 1))) void k_terms_vjp(DevPlan<T> d) {
  using K = Kern<T, P, E>;
  constexpr unsigned S = sizeof(T);
  __shared__ T smem[K::LDS];
  Fft2<T, P, E> eng;
  setup(eng, smem, d.tw);
  const int cell = blockIdx.x / kTermsVjpTasks;
  const int task = blockIdx.x % kTermsVjpTasks;
  const unsigned vo = threadIdx.x * S;
  const rsrc_t rs = mkbuf(d.spec + (size_t)cell * 8 * K::FSZ, 8 * K::FSZ);
  const rsrc_t rw = mkbuf(d.wP + (size_t)cell * 5 * K::FSZ, 5 * K::FSZ);
  const rsrc_t ra = mkbuf(d.acot + (size_t)cell * 16 * K::FSZ, 16 * K::FSZ);
  const size_t tabn = (size_t)d.J * K::FSZ;
  if (task < 7) {
    const int g = task < 3 ? task + 1 : task - 3;
    const bool odd = task < 3;
    const rsrc_t rin = mkbuf(odd ? d.phip : d.psip, tabn);
    const rsrc_t rout = mkbuf(odd ? d.Kt : d.psiw, tabn);
    const rsrc_t rd = mkbuf(d.acc + ((size_t)cell * 7 + task) * 2 * K::FSZ, 2 * K::FSZ);
    const rsrc_t rc = mkbuf(d.fwa + ((size_t)cell * 7 + task) * 2 * K::FSZ, 2 * K::FSZ);
    const rsrc_t rf = mkbuf(d.gf0 + ((size_t)cell * 7 + task) * K::FSZ, K::FSZ);
    const rsrc_t rg = mkbuf(d.gspec + ((size_t)cell * 11 + task) * 2 * K::FSZ, 2 * K::FSZ);
    const rsrc_t ro = mkbuf(d.terms + ((size_t)cell * kTermPlanes + task) * K::FSZ, K::FSZ);
    const unsigned fg = 2 * g * K::FSZ;
    const T sgn = odd ? (T)-1 : (T)1;
    {
      // D = F field_bar for the real field_bar (d = conj D)
      T zr[E], zi[E];
#pragma unroll
      for (int n = 0; n < E; ++n) {
        zr[n] = bld<T>(ra, vo, (task * K::FSZ + n * K::NT) * S);
        zi[n] = 0;
      }
      eng.fwd2(zr, zi);
#pragma unroll
      for (int k = 0; k < E; ++k) {
        bst<T>(rd, zr[k], vo, (k * K::NT) * S);
        bst<T>(rd, zi[k], vo, (K::FSZ + k * K::NT) * S);
      }
    }
#pragma unroll 1
    for (int j = 0; j < d.J; j += 2) {
      const unsigned t1 = j * K::FSZ, t2 = t1 + K::FSZ;
      // B stays in registers for its two uses (some go to scratch under the
      // 128-register cap; measured 4 % faster than a per-task buffer)
      T zr[E], zi[E], Br[E], Bi[E];
      // B = inv2(cb D) = b_j + i b_j+1 up to the phase
#pragma unroll
      for (int k = 0; k < E; ++k) {
        const unsigned o = k * K::NT;
        const T o1 = bld<T>(rout, vo, (t1 + o) * S), o2 = bld<T>(rout, vo, (t2 + o) * S);
        const T cr = odd ? -o2 : o1, ci = odd ? o1 : o2;
        const T dr = bld<T>(rd, vo, o * S), di = bld<T>(rd, vo, (K::FSZ + o) * S);
        zr[k] = cr * dr - ci * di;
        zi[k] = cr * di + ci * dr;
      }
      eng.inv2(zr, zi);
#pragma unroll
      for (int n = 0; n < E; ++n) {
        Br[n] = zr[n];
        Bi[n] = zi[n];
      }
      // A = inv2(cin w_hat_g) = a_j + i a_j+1 up to the phase
#pragma unroll
      for (int k = 0; k < E; ++k) {
        const unsigned o = k * K::NT;
        const T i1 = bld<T>(rin, vo, (t1 + o) * S), i2 = bld<T>(rin, vo, (t2 + o) * S);
        const T cr = odd ? i2 : i1, ci = odd ? -i1 : i2;
        const T sr = bld<T>(rs, vo, (fg + o) * S), si = bld<T>(rs, vo, (fg + K::FSZ + o) * S);
        zr[k] = sr * cr - si * ci;
        zi[k] = sr * ci + si * cr;
      }
      eng.inv2(zr, zi);
#pragma unroll
      for (int n = 0; n < E; ++n) {
        const unsigned o = n * K::NT;
        const T br = Br[n], bi = Bi[n];
        const T f0 = bld<T>(rw, vo, (4 * K::FSZ + o) * S);
        T fb = sgn * (zr[n] * br + zi[n] * bi);
        if (j != 0) fb += bld<T>(rf, vo, o * S);
        bst<T>(rf, fb, vo, o * S);
        // forward: f0 A, transformed by fwd2 below
        zr[n] *= f0;
        zi[n] *= f0;
      }
      // the pair's forward contribution cout fwd2(f0 A)
      eng.fwd2(zr, zi);
#pragma unroll
      for (int k = 0; k < E; ++k) {
        const unsigned o = k * K::NT;
        const T o1 = bld<T>(rout, vo, (t1 + o) * S), o2 = bld<T>(rout, vo, (t2 + o) * S);
        const T cr = odd ? o2 : o1, ci = odd ? o1 : -o2;
        T ar = cr * zr[k] - ci * zi[k], ai = cr * zi[k] + ci * zr[k];
        // read at j = 0 too (not yet written) and dropped by a select
        const T pr = bld<T>(rc, vo, o * S), pi = bld<T>(rc, vo, (K::FSZ + o) * S);
        ar += j != 0 ? pr : (T)0;
        ai += j != 0 ? pi : (T)0;
        bst<T>(rc, ar, vo, o * S);
        bst<T>(rc, ai, vo, (K::FSZ + o) * S);
      }
      // Z = fwd2(f0 B);  H += cw conj(Z)
#pragma unroll
      for (int n = 0; n < E; ++n) {
        const unsigned o = n * K::NT;
        const T f0 = bld<T>(rw, vo, (4 * K::FSZ + o) * S);
        zr[n] = f0 * Br[n];
        zi[n] = f0 * Bi[n];
      }
      eng.fwd2(zr, zi);
#pragma unroll
      for (int k = 0; k < E; ++k) {
        const unsigned o = k * K::NT;
        const T i1 = bld<T>(rin, vo, (t1 + o) * S), i2 = bld<T>(rin, vo, (t2 + o) * S);
        const T cr = odd ? -i2 : i1, ci = odd ? i1 : i2;
        T xr = cr * zr[k] + ci * zi[k], xi = ci * zr[k] - cr * zi[k];
        if (j != 0) {
          xr += bld<T>(rg, vo, o * S);
          xi += bld<T>(rg, vo, (K::FSZ + o) * S);
        }
        bst<T>(rg, xr, vo, o * S);
        bst<T>(rg, xi, vo, (K::FSZ + o) * S);
      }
    }
    // the forward field: Re inv2(sum over pairs)
    T zr[E], zi[E];
#pragma unroll
    for (int k = 0; k < E; ++k) {
      const unsigned o = k * K::NT;
      zr[k] = bld<T>(rc, vo, o * S);
      zi[k] = bld<T>(rc, vo, (K::FSZ + o) * S);
    }
    eng.inv2(zr, zi);
#pragma unroll
    for (int n = 0; n < E; ++n) bst<T>(ro, zr[n], vo, (n * K::NT) * S);
  } else {
    const T wj = (T)(kPi / d.J);
    const rsrc_t rps = mkbuf(d.psi, tabn);
    const rsrc_t rpp = mkbuf(d.psip, tabn);
    const int mu = task - 7;
    const unsigned fm = 2 * mu * K::FSZ;
    const rsrc_t rg = mkbuf(d.gspec + ((size_t)cell * 11 + 7 + mu) * 2 * K::FSZ, 2 * K::FSZ);
    const rsrc_t rsp = mkbuf(d.terms + ((size_t)cell * kTermPlanes + task) * K::FSZ, K::FSZ);
    const T e = mu == 0 ? wj : -wj;
    T Sacc[E];
#pragma unroll
    for (int n = 0; n < E; ++n) Sacc[n] = 0;
#pragma unroll 1
    for (int j = 0; j < d.J; ++j) {
      const unsigned tj = j * K::FSZ;
      T zr[E], zi[E];
#pragma unroll
      for (int k = 0; k < E; ++k) {
        const unsigned o = k * K::NT;
        const T ar = bld<T>(rs, vo, (fm + o) * S), ai = bld<T>(rs, vo, (fm + K::FSZ + o) * S);
        const T a = bld<T>(rps, vo, (tj + o) * S), b = bld<T>(rpp, vo, (tj + o) * S);
        zr[k] = ar * a - ai * b;
        zi[k] = ai * a + ar * b;
      }
      eng.inv2(zr, zi);  // (A, B)
#pragma unroll
      for (int n = 0; n < E; ++n) {
        Sacc[n] += e * zr[n] * zi[n];  // the forward accumulator's share
        const T sb = e * bld<T>(ra, vo, (7 * K::FSZ + n * K::NT) * S);
        const T A = zr[n];
        zr[n] = sb * zi[n];  // S_bar e B
        zi[n] = sb * A;      // S_bar e A
      }
      eng.fwd2(zr, zi);
#pragma unroll
      for (int k = 0; k < E; ++k) {
        const unsigned o = k * K::NT;
        const T a = bld<T>(rps, vo, (tj + o) * S), b = bld<T>(rpp, vo, (tj + o) * S);
        T xr = a * zr[k] + b * zi[k], xi = b * zr[k] - a * zi[k];
        if (j != 0) {
          xr += bld<T>(rg, vo, o * S);
          xi += bld<T>(rg, vo, (K::FSZ + o) * S);
        }
        bst<T>(rg, xr, vo, o * S);
        bst<T>(rg, xi, vo, (K::FSZ + o) * S);
      }
    }
#pragma unroll
    for (int n = 0; n < E; ++n) bst<T>(rsp, Sacc[n], vo, (n * K::NT) * S);
  }
}

// ------------------------------------------------------------------ I_3
// Transpose of k_i3, one workgroup per (cell, j), Gauss-Legendre nodes in
// symmetric pairs (m, m' = M-1-m; the middle node of an odd M alone).
// With S the shift of node m, s_nu = S w_nu, b_bar the cotangent of the I_3
// sums (b_bar_0 = -2 pi lam_0, b_bar_k = 2 pi lam_k), t_nu = S b_bar_nu,
// Psi = inv2(psi'_j / P^2 fwd2(.)) (real, symmetric) and c = (pi/J) w_m,
// the forward pair contributes
//   c sum_{a,nu} < eta_a b_bar_nu s_a + eta_nu t_a w_nu , q_a,nu >,
//   q_a,nu = Psi(w_a s_nu)
// to the loss (node m through s_a, node m' through S^{-1} = S^T acting on
// its partner sums).  Its derivative has two parts:
//   * the factors beside q, with q fixed:
//       Y_a      += c eta_a sum_nu b_bar_nu q_a,nu    (Y: cotangent of s)
//       w_bar_nu += c eta_nu sum_a t_a q_a,nu
//   * q through Psi, which is symmetric: with R_a,nu = Psi(T_a,nu),
//     T_a,nu = eta_a b_bar_nu s_a + eta_nu t_a w_nu,
//       w_bar_a  += c sum_nu s_nu R_a,nu
//       Y_nu     += c sum_a w_a R_a,nu
//   w_hat_bar += phase conj(F)(Y)        (S transposed, per node pair)
// The two terms of T are summed before the convolution because Psi is
// linear and both pair with the same variation of w_a s_nu: one family
// R replaces the separate convolutions of b_bar_nu s_a and t_a w_nu.  Per
// node pair: 4 shift transforms, 2 x 8 packed convolutions of 2
// transforms, 2 final transforms (38, against 20 in the forward kernel).
// For rows (a0, a1) the loop over nu runs q and R back to back, so Y_a
// and, with WREG, w_bar_a accumulate in registers; w_bar_nu and Y_nu go
// through memory once per convolution.  Where the register budget of the
// tile allows (RREG), the rows' own fields s_a0, s_a1, t_a0, t_a1 are also
// loaded into registers once per row pair instead of once per convolution.
// The tuner picks WREG: the extra registers cost occupancy.
// i3g[cell][j]: [0..3] w_bar (row real), [4..7] w_hat_bar packed as
// (mu 0 + i mu 1), (mu 2 + i mu 3), re/im planes, col spec.
template <typename T, int P, int E, bool WREG>
__global__ __launch_bounds__((Fft2<T, P, E>::NT)) void k_i3_vjp_reg(DevPlan<T> d, int ncells) {
  using K = Kern<T, P, E, true>;
  constexpr unsigned S = sizeof(T);
  // elements between scheduling barriers in the element loops, which bound
  // the loads in flight
#ifndef QB_VJP_SG
#define QB_VJP_SG 4
#endif
  constexpr int SG = QB_VJP_SG;
  // registers: the transform operand, Y of the rows, w_bar of the rows
  // (WREG) and the rows' four shifted fields (RREG), E values each per
  // field and thread, beside about 48 for addresses and temporaries
  constexpr int F = I3Regs<T, P, E>::F;
  constexpr bool RREG = 2 * F + 2 * F + (WREG ? 2 * F : 0) + 4 * F + 48 <= I3Regs<T, P, E>::BUDGET;
  constexpr int RE = RREG ? E : 1;
  // Two fields of LDS beside the transpose buffer, where they fit and the
  // workgroup fills its compute unit anyway (512 threads or more): three
  // private reads per nu (the old w_bar_nu
  // before the q convolution, the old Y_nu and s_nu before the R
  // convolution) are copied there by buffer-to-LDS loads issued before the
  // convolution, so their latency hides behind its transforms.
  constexpr bool STG = K::NT >= 512 && (K::LDS + 2 * K::FSZ) * (int)sizeof(T) <= 160 * 1024;
  constexpr int PFD = STG ? K::FSZ * (int)sizeof(T) / 4 : 1;  // dwords of one staged field
  __shared__ unsigned pfs[STG ? 2 * PFD : 1];
  __shared__ T smem[K::LDS];
  typename K::Eng eng;
  setup(eng, smem, d.tw);
  const int task = xcd_task(blockIdx.x, gridDim.x);
  const int cell = task / d.J;
  const int j = task % d.J;
  const unsigned vo = threadIdx.x * S;
  const size_t tb = (size_t)cell * d.J + j;
  const rsrc_t rs = mkbuf(d.spec + (size_t)cell * 8 * K::FSZ, 8 * K::FSZ);
  const rsrc_t rw = mkbuf(d.wP + (size_t)cell * 5 * K::FSZ, 5 * K::FSZ);
  const rsrc_t rl = mkbuf(d.acot + ((size_t)cell * 16 + 8) * K::FSZ, 4 * K::FSZ);
  const rsrc_t rh = mkbuf(d.lamh + (size_t)cell * 4 * K::FSZ, 4 * K::FSZ);
  const rsrc_t rg = mkbuf(d.i3g + tb * 8 * K::FSZ, 8 * K::FSZ);
  const rsrc_t rb = mkbuf(d.i3s + tb * 4 * K::FSZ, 4 * K::FSZ);
  const rsrc_t rt = mkbuf(d.i3t + tb * 4 * K::FSZ, 4 * K::FSZ);
  const rsrc_t rc = mkbuf(d.i3sb + tb * 4 * K::FSZ, 4 * K::FSZ);
  const rsrc_t rm = mkbuf(d.psips + (size_t)j * K::FSZ, K::FSZ);
  const int kx = eng.line;
  // i3g planes 0..3 start at zero: with WREG their first touch is the q
  // consumer of the first row pair (a select drops the old value); without
  // it the R consumer touches a1 first, so they are cleared here.  Planes
  // 4..7 take their first values at the first node pair (a select again).
  if constexpr (!WREG) {
#pragma unroll 1
    for (int q = 0; q < 4; ++q)
#pragma unroll
      for (int n = 0; n < E; ++n) bst<T>(rg, (T)0, vo, (q * K::FSZ + n * K::NT) * S);
  }
  auto conv = [&](T (&zr)[E], T (&zi)[E]) {
    eng.fwd2(zr, zi);
#pragma unroll
    for (int k = 0; k < E; ++k) {
      const T a = bld<T>(rm, vo, (k * K::NT) * S);
      zr[k] *= a;
      zi[k] *= a;
    }
    eng.inv2(zr, zi);
  };
  auto ld = [&](rsrc_t r, int plane, unsigned o) { return bld<T>(r, vo, (plane * K::FSZ + o) * S); };
  auto rmw = [&](rsrc_t r, int plane, unsigned o, T v) {
    const unsigned off = (plane * K::FSZ + o) * S;
    bst<T>(r, bld<T>(r, vo, off) + v, vo, off);
  };
  const int nnode = (d.M + 1) / 2;
#pragma unroll 1
  for (int m = 0; m < nnode; ++m) {
    const bool paired = m != d.M - 1 - m;
    const T* px = d.phx + (((size_t)j * d.M + m) * P) * 2;
    const T* py = d.phy + (((size_t)j * d.M + m) * P) * 2 + 2 * E * eng.bq;
    const T pxr = px[2 * kx], pxi = px[2 * kx + 1];
    // s_nu = S w_nu, and t_nu = S b_bar_nu (zero for an unpaired node: its
    // partner terms vanish), two packed shifts each
#pragma unroll 1
    for (int src = 0; src < 2; ++src) {
#pragma unroll 1
      for (int pr = 0; pr < 2; ++pr) {
        T zr[E], zi[E];
        const rsrc_t rd = src == 0 ? rb : rt;
        if (src == 1 && !paired) {
#pragma unroll
          for (int n = 0; n < E; ++n) {
            bst<T>(rd, (T)0, vo, ((2 * pr) * K::FSZ + n * K::NT) * S);
            bst<T>(rd, (T)0, vo, ((2 * pr + 1) * K::FSZ + n * K::NT) * S);
          }
          continue;
        }
#pragma unroll
        for (int k = 0; k < E; ++k) {
          const unsigned o = k * K::NT;
          T er, ei;
          cmul(pxr, pxi, py[2 * k], py[2 * k + 1], er, ei);
          if (src == 0) {
            const unsigned fa = 2 * (2 * pr) * K::FSZ, fb = 2 * (2 * pr + 1) * K::FSZ;
            T ar, ai, br, bi;
            cmul(bld<T>(rs, vo, (fa + o) * S), bld<T>(rs, vo, (fa + K::FSZ + o) * S), er, ei, ar, ai);
            cmul(bld<T>(rs, vo, (fb + o) * S), bld<T>(rs, vo, (fb + K::FSZ + o) * S), er, ei, br, bi);
            zr[k] = ar - bi;
            zi[k] = ai + br;
          } else {
            cmul(ld(rh, 2 * pr, o), ld(rh, 2 * pr + 1, o), er, ei, zr[k], zi[k]);
          }
        }
        eng.inv2(zr, zi);
        // t carries the B-term factors of b_bar: -2 pi (mu = 0), 2 pi (mu > 0)
        const T fa = src == 0 ? (T)1 : (T)(pr == 0 ? -2.0 * kPi : 2.0 * kPi);
        const T fb = src == 0 ? (T)1 : (T)(2.0 * kPi);
#pragma unroll
        for (int n = 0; n < E; ++n) {
          bst<T>(rd, fa * zr[n], vo, ((2 * pr) * K::FSZ + n * K::NT) * S);
          bst<T>(rd, fb * zi[n], vo, ((2 * pr + 1) * K::FSZ + n * K::NT) * S);
        }
      }
    }
    // Y (the S-transposed cotangent of this node pair) is first written by
    // the first row pair's convolutions (every column nu), then accumulated
    const T c = d.wm[m];
#pragma unroll 1
    for (int mp = 0; mp < 2; ++mp) {
      const int a0 = 2 * mp, a1 = 2 * mp + 1;
      const bool first = m == 0 && mp == 0;
      const T ea0 = a0 == 0 ? (T)1 : (T)-1;  // eta_a0; eta_a1 = -1
      T ya0[E], ya1[E], wa0[WREG ? E : 1], wa1[WREG ? E : 1];
#pragma unroll
      for (int n = 0; n < E; ++n) ya0[n] = ya1[n] = 0;
      if constexpr (WREG) {
#pragma unroll
        for (int n = 0; n < E; ++n) wa0[WREG ? n : 0] = wa1[WREG ? n : 0] = 0;
      }
      // the rows' shifted fields s_a, t_a (registers with RREG)
      T sa0[RE], sa1[RE], ta0[RE], ta1[RE];
      if constexpr (RREG) {
#pragma unroll
        for (int n = 0; n < E; ++n) {
          const unsigned o = n * K::NT;
          sa0[RREG ? n : 0] = ld(rb, a0, o);
          sa1[RREG ? n : 0] = ld(rb, a1, o);
          ta0[RREG ? n : 0] = ld(rt, a0, o);
          ta1[RREG ? n : 0] = ld(rt, a1, o);
        }
      }
      auto row = [&](const T (&r)[RE], rsrc_t buf, int plane, int n) {
        if constexpr (RREG)
          return r[RREG ? n : 0];
        else
          return ld(buf, plane, n * K::NT);
      };
      // The element loops are fused across the two convolutions of a nu:
      // consuming q also builds the input of R (b_bar_nu is loaded once),
      // and consuming R builds the input of the next nu's q (w_a0, w_a1
      // are loaded once per nu).
      T zr[E], zi[E];
#pragma unroll
      for (int n = 0; n < E; ++n) {
        const unsigned o = n * K::NT;
        const T sv = ld(rb, 0, o);
        zr[n] = ld(rw, a0, o) * sv;
        zi[n] = ld(rw, a1, o) * sv;
        if (n % SG == SG - 1) __builtin_amdgcn_sched_barrier(0);
      }
#pragma unroll 1
      for (int nu = 0; nu < 4; ++nu) {
        const T enu = nu == 0 ? (T)1 : (T)-1;  // eta_nu
        // q_a,nu = Psi(w_a s_nu); then R_a,nu = Psi(eta_a b_bar_nu s_a + eta_nu t_a w_nu)
        if constexpr (STG) fetch_lds_dw<T, K::NT, E>(rg, pfs, vo, nu * K::FSZ * S);
        conv(zr, zi);
        const unsigned pq = STG ? lds_fetch_wait() : 0u;
#pragma unroll
        for (int n = 0; n < E; ++n) {
          const unsigned o = n * K::NT;
          const T b = ld(rl, nu, o), bb = c * b;
          const T ta0v = row(ta0, rt, a0, n), ta1v = row(ta1, rt, a1, n);
          ya0[n] += ea0 * bb * zr[n];
          ya1[n] -= bb * zi[n];
          const T gv = enu * c * (ta0v * zr[n] + ta1v * zi[n]);
          {
            const T gp = STG ? lds_elem<T, K::NT, E>(pfs, n, pq) : bld<T>(rg, vo, (nu * K::FSZ + o) * S);
            bst<T>(rg, gv + (WREG && first ? (T)0 : gp), vo, (nu * K::FSZ + o) * S);
          }
          const T wv = enu * ld(rw, nu, o);
          zr[n] = ea0 * b * row(sa0, rb, a0, n) + wv * ta0v;
          zi[n] = wv * ta1v - b * row(sa1, rb, a1, n);
          if (n % SG == SG - 1) __builtin_amdgcn_sched_barrier(0);
        }
        if constexpr (STG) {
          fetch_lds_dw<T, K::NT, E>(rc, pfs, vo, nu * K::FSZ * S);
          fetch_lds_dw<T, K::NT, E>(rb, pfs + PFD, vo, nu * K::FSZ * S);
        }
        conv(zr, zi);
        const unsigned pr2 = STG ? lds_fetch_wait() : 0u;
        // next q input: s of the next nu (re-read on the last pass, unused)
        const int nx = nu < 3 ? nu + 1 : 3;
#pragma unroll
        for (int n = 0; n < E; ++n) {
          const unsigned o = n * K::NT;
          const T sv = c * (STG ? lds_elem<T, K::NT, E>(pfs + PFD, n, pr2) : ld(rb, nu, o));
          if constexpr (WREG) {
            wa0[WREG ? n : 0] += sv * zr[n];
            wa1[WREG ? n : 0] += sv * zi[n];
          } else {
            rmw(rg, a0, o, sv * zr[n]);
            rmw(rg, a1, o, sv * zi[n]);
          }
          const T w0 = ld(rw, a0, o), w1 = ld(rw, a1, o);
          // first row pair: the old value is read (in bounds) but dropped by
          // a select, which keeps the loop free of branches
          const unsigned yo = (nu * K::FSZ + o) * S;
          const T yp = STG ? lds_elem<T, K::NT, E>(pfs, n, pr2) : bld<T>(rc, vo, yo);
          bst<T>(rc, c * (w0 * zr[n] + w1 * zi[n]) + (mp != 0 ? yp : (T)0), vo, yo);
          const T sn = ld(rb, nx, o);
          zr[n] = w0 * sn;
          zi[n] = w1 * sn;
          if (n % SG == SG - 1) __builtin_amdgcn_sched_barrier(0);
        }
      }
#pragma unroll
      for (int n = 0; n < E; ++n) {
        const unsigned o = n * K::NT;
        rmw(rc, a0, o, ya0[n]);
        rmw(rc, a1, o, ya1[n]);
        if constexpr (WREG) {
          rmw(rg, a0, o, wa0[WREG ? n : 0]);
          rmw(rg, a1, o, wa1[WREG ? n : 0]);
        }
      }
    }
    // w_hat_bar += phase conj(F)(Y), packed pairs (0, 1), (2, 3).  Only its
    // entries on Xi are read back (k_grad_out keeps Xi and drops the rest
    // with a select), so the other lanes' accesses get an offset past the
    // buffer (loads 0, stores dropped) and those entries are never written.
    const int bx = centered<P>(kx);
    const bool kx_in = bx > -P / 4 && bx < P / 4;
#pragma unroll 1
    for (int pr = 0; pr < 2; ++pr) {
      T zr[E], zi[E];
#pragma unroll
      for (int n = 0; n < E; ++n) {
        const unsigned o = n * K::NT;
        zr[n] = ld(rc, 2 * pr, o);
        zi[n] = -ld(rc, 2 * pr + 1, o);
      }
      eng.fwd2(zr, zi);
#pragma unroll
      for (int k = 0; k < E; ++k) {
        const unsigned o = k * K::NT;
        const int by = centered<P>(eng.bk(k));
        const unsigned vk = (kx_in && by > -P / 4 && by < P / 4) ? vo : 0x80000000u;
        T er, ei;
        cmul(pxr, pxi, py[2 * k], py[2 * k + 1], er, ei);
        T xr, xi;
        cmul(zr[k], -zi[k], er, ei, xr, xi);
        const unsigned fr = ((4 + 2 * pr) * K::FSZ + o) * S, fi = ((5 + 2 * pr) * K::FSZ + o) * S;
        const T g0 = bld<T>(rg, vk, fr), g1 = bld<T>(rg, vk, fi);
        bst<T>(rg, xr + (m != 0 ? g0 : (T)0), vk, fr);
        bst<T>(rg, xi + (m != 0 ? g1 : (T)0), vk, fi);
      }
    }
  }
}

// ------------------------------------------------------------------ gradient on the grid
// Elementwise gathering of every cotangent of the interpolants and of
// w_hat into gsum[cell][8] (flat index e, the same in both layouts):
//   q = 0..3  total real-space cotangent of w_mu on the P grid (row real):
//             the I_3 partials summed over j, the assembly's explicit part,
//             and 2 f0_bar for mu = 0
//   q = 4..7  w_hat cotangents packed as (mu 0 + i mu 1), (mu 2 + i mu 3),
//             re / im planes (col spec): the I_3 partials summed over j and
//             the single-component spectra of the I_1, I_4 and I_2 tasks.
template <typename T>
__global__ void k_grad_pre(DevPlan<T> d, int ncells, int fsz) {
  const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const size_t per = (size_t)8 * fsz;
  if (idx >= (size_t)ncells * per) return;
  const size_t cell = idx / per, r = idx % per;
  const int q = (int)(r / fsz);
  const size_t e = r % fsz;
  const T* src = d.i3g + cell * d.J * per + r;
  T a = 0;
  for (int j = 0; j < d.J; ++j) a += src[(size_t)j * per];
  if (q < 4) {
    a += d.acot[(cell * 16 + 12 + q) * fsz + e];
    if (q == 0) {
      T f = 0;
      for (int t = 0; t < 7; ++t) f += d.gf0[(cell * 7 + t) * fsz + e];
      a += (T)2 * f;
    }
  } else {
    const int pr = (q - 4) / 2, im = (q - 4) % 2;
    const int ma = 2 * pr, mb = 2 * pr + 1;
    // task slots of gspec: I_1 (mu >= 1) at mu - 1, I_4 at 3 + mu, I_2 at 7 + mu
    // k_terms_vjp leaves H with the cotangent (H(k) + conj H(-k)) / 2
    const T* gs = d.gspec + cell * 22 * fsz + e;
    const T* gn = d.gspec + cell * 22 * fsz + d.negk[e];
    T ar = 0, ai = 0, br = 0, bi = 0;
    const int sa[3] = {ma - 1, 3 + ma, 7 + ma}, sb[3] = {mb - 1, 3 + mb, 7 + mb};
    for (int t = 0; t < 3; ++t) {
      if (sa[t] >= 0) {
        ar += gs[(size_t)(2 * sa[t]) * fsz] + gn[(size_t)(2 * sa[t]) * fsz];
        ai += gs[(size_t)(2 * sa[t] + 1) * fsz] - gn[(size_t)(2 * sa[t] + 1) * fsz];
      }
      br += gs[(size_t)(2 * sb[t]) * fsz] + gn[(size_t)(2 * sb[t]) * fsz];
      bi += gs[(size_t)(2 * sb[t] + 1) * fsz] - gn[(size_t)(2 * sb[t] + 1) * fsz];
    }
    a += (T)0.5 * (im == 0 ? ar - bi : ai + br);
  }
  d.gsum[cell * per + r] = a;
}

// Transpose of k_dft_in: adds conj(F) of the total real-space cotangent of
// the P-grid interpolants to the spectral cotangents (both from k_grad_pre),
// keeps Xi without its -N/2 rows and columns, scales by 1/N^2 and applies F
// at the even points:
//   w_bar(n) = Re sum_{xi} w_hat_bar(xi) e^{-2 pi i xi . n / N} / N^2.
template <typename T, int P, int E>
__global__ __launch_bounds__((Fft2<T, P, E>::NT)) void k_grad_out(DevPlan<T> d, T* __restrict__ gout, int cell0) {
  using K = Kern<T, P, E>;
  constexpr unsigned S = sizeof(T);
  __shared__ T smem[K::LDS];
  Fft2<T, P, E> eng;
  setup(eng, smem, d.tw);
  const int lc = blockIdx.x;
  const int cell = cell0 + lc;
  const int N = P / 2;
  const unsigned vo = threadIdx.x * S;
  const size_t cs = (size_t)d.Nx * N * N;
  const rsrc_t r3 = mkbuf(d.gsum + (size_t)lc * 8 * K::FSZ, 8 * K::FSZ);
  const int bx = centered<P>(eng.line);
  const bool kx_in = bx > -N / 2 && bx < N / 2;
  const T sc = (T)1 / (T)(N * N);
#pragma unroll 1
  for (int pr = 0; pr < 2; ++pr) {
    const int ma = 2 * pr, mb = 2 * pr + 1;
    T zr[E], zi[E];
#pragma unroll
    for (int n = 0; n < E; ++n) {
      const unsigned o = n * K::NT;
      zr[n] = bld<T>(r3, vo, (ma * K::FSZ + o) * S);
      zi[n] = -bld<T>(r3, vo, (mb * K::FSZ + o) * S);
    }
    eng.fwd2(zr, zi);  // conj(F)(a + i b) = conj(fwd2(a - i b))
#pragma unroll
    for (int k = 0; k < E; ++k) {
      const unsigned o = k * K::NT;
      T Zr = zr[k] + bld<T>(r3, vo, ((4 + 2 * pr) * K::FSZ + o) * S);
      T Zi = -zi[k] + bld<T>(r3, vo, ((5 + 2 * pr) * K::FSZ + o) * S);
      const int by = centered<P>(eng.bk(k));
      const bool in = kx_in && by > -N / 2 && by < N / 2;
      // F applied below as conj(inv2(conj Z))
      zr[k] = in ? Zr * sc : (T)0;
      zi[k] = in ? -Zi * sc : (T)0;
    }
    eng.inv2(zr, zi);
    const int y = eng.line;
    if (((eng.q | y) & 1) == 0) {
      T* ga = gout + ma * cs + (size_t)cell * N * N + (centered<P>(y) / 2 + N / 2);
      T* gb = ga + cs;
#pragma unroll
      for (int n = 0; n < E; ++n) {
        const int i = vel_index<P, K::TPR>(eng.q, n);
        ga[i * N] = zr[n];
        gb[i * N] = -zi[n];
      }
    }
  }
}

// ------------------------------------------------------------------ transport
// Cotangent of the ghost-extended state, ext index k in [0, Nx + 4) (cell
// k - 2), for the step out_c = W0 + dt/(2dx) (-v (Wp - Wm) + |v| (Wp - 2 W0
// + Wm) + lim (-v (Sp - Sm) + |v| (Sp - 2 S0 + Sm))) with
// S_k = minmod(d_k, d_{k-1}), d_k = we_{k+1} - we_k, and the limiter
// branches taken at the forward state w.
template <typename T>
__global__ void k_transport_vjp_ext(const T* __restrict__ w, const T* __restrict__ lam, T* __restrict__ ext,
                                    const T* __restrict__ bcw, const double* __restrict__ flux, BcDev bl,
                                    BcDev br, T dt, int Nx, int N, T L) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  const int per = N * N;
  const int NE = Nx + 4;
  if (idx >= NE * per) return;
  const int k = idx / per;
  const int e = idx % per;
  const int i = e / N;
  const T h = (T)2 * L / (T)N;
  const T vx = h * (T)(i - N / 2);
  const T dx = (T)1 / (T)Nx;
  const size_t cs = (size_t)Nx * per;
  const T c = dt / ((T)2 * dx);
  const T nu = dt * vx / dx;
  const T sg = vx > (T)0 ? (T)1 : (vx < (T)0 ? (T)-1 : (T)0);
  const T lim = (T)0.5 * (sg - nu);
  const T av = fabs(vx);
  for (int mu = 0; mu < 4; ++mu) {
    // we at ext k-2 .. k+2 and lam at out cells k-4 .. k
    T we[5], la[5];
    for (int o = 0; o < 5; ++o) {
      const int kk = k - 2 + o;
      we[o] = (kk >= 0 && kk < NE) ? ext_value(w, bcw, flux, bl, br, mu, kk - 2, e, i, vx, Nx, N, cs) : (T)0;
      const int oc = k - 4 + o;
      la[o] = (oc >= 0 && oc < Nx) ? lam[mu * cs + (size_t)oc * per + e] : (T)0;
    }
    // lam_S at ext kappa = k - 1 + t, t = 0..2: uses lam(kappa-3..kappa-1) = la[t .. t+2]
    T lS[3];
    bool pa[3], pb[3];
    for (int t = 0; t < 3; ++t) {
      const int kap = k - 1 + t;
      const bool valid = kap >= 1 && kap <= Nx + 2;
      lS[t] = valid ? c * lim * ((-vx + av) * la[t] + (vx + av) * la[t + 2] - (T)2 * av * la[t + 1]) : (T)0;
      const T a = we[t + 2] - we[t + 1], b = we[t + 1] - we[t];
      const bool pos = valid && a * b > (T)0;
      const bool le = fabs(a) <= fabs(b);
      pa[t] = pos && le;
      pb[t] = pos && !le;
    }
    // lam_d at kappa = k - 1 (t = 0) and k (t = 1)
    const T ldm = (pa[0] ? lS[0] : (T)0) + (pb[1] ? lS[1] : (T)0);
    const T ld0 = (pa[1] ? lS[1] : (T)0) + (pb[2] ? lS[2] : (T)0);
    T r = ((T)1 - (T)2 * c * av) * la[2] + c * (-vx + av) * la[1] + c * (vx + av) * la[3];
    if (k >= 1) r += ldm;
    if (k <= Nx + 2) r -= ld0;
    ext[(size_t)mu * NE * per + (size_t)k * per + e] = r;
  }
}

// Maxwell walls: alpha / Z * sum over inflow rows of <ghost cotangent, W_FD>
// (float64), the cotangent of the outgoing flux Fbar.  One workgroup per wall.
template <typename T>
__global__ void k_maxwell_lflux(const T* __restrict__ ext, const T* __restrict__ bcw, double* __restrict__ lflux,
                                BcDev bl, BcDev br, int Nx, int N) {
  const int wall = blockIdx.x;
  const BcDev& bc = wall == 0 ? bl : br;
  if (bc.kind != 2) return;
  const int per = N * N;
  const int NE = Nx + 4;
  const int g0 = wall == 0 ? 0 : Nx + 2;
  double s = 0.0;
  for (int e = threadIdx.x; e < per; e += blockDim.x) {
    const int i = e / N;
    const bool inflow = wall == 0 ? (i > N / 2) : (i < N / 2 && i != 0);
    if (!inflow) continue;
    for (int mu = 0; mu < 4; ++mu) {
      const double fd = (double)bcw[(size_t)wall * 4 * per + (size_t)mu * per + e];
      const size_t b = (size_t)mu * NE * per + e;
      s += fd * ((double)ext[b + (size_t)g0 * per] + (double)ext[b + (size_t)(g0 + 1) * per]);
    }
  }
  __shared__ double red[256];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int o = blockDim.x / 2; o > 0; o >>= 1) {
    if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) lflux[wall] = bc.alpha / bc.Z * red[0];
}

// Fold the ghost cotangents back onto the cells (transpose of the ghost rule).
template <typename T>
__global__ void k_transport_vjp_fold(const T* __restrict__ ext, T* __restrict__ out, const double* __restrict__ lflux,
                                     BcDev bl, BcDev br, int Nx, int N, T L) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  const int per = N * N;
  if (idx >= Nx * per) return;
  const int NE = Nx + 4;
  const int c = idx / per;
  const int e = idx % per;
  const int i = e / N, col = e % N;
  const double h = 2.0 * (double)L / N;
  const double vx = h * (i - N / 2);
  const size_t cs = (size_t)Nx * per;
  for (int mu = 0; mu < 4; ++mu) {
    const T* x = ext + (size_t)mu * NE * per;
    T acc = x[(size_t)(c + 2) * per + e];
    if (bl.kind == 0) {
      const int gk[4] = {0, 1, Nx + 2, Nx + 3};
      for (int t = 0; t < 4; ++t)
        if ((((gk[t] - 2) % Nx) + Nx) % Nx == c) acc += x[(size_t)gk[t] * per + e];
    } else {
      for (int wall = 0; wall < 2; ++wall) {
        const int cell = wall == 0 ? 0 : Nx - 1;
        if (c != cell) continue;
        const BcDev& bc = wall == 0 ? bl : br;
        const int g0 = wall == 0 ? 0 : Nx + 2;
        auto inflow = [&](int row) {
          return wall == 0 ? (row > N / 2) : (row < N / 2 && !(bc.kind == 2 && row == 0));
        };
        if (!inflow(i)) acc += x[(size_t)g0 * per + e] + x[(size_t)(g0 + 1) * per + e];
        if (bc.kind == 2) {
          const int r = N - i;  // the inflow row whose mirror is row i
          if (i >= 1 && inflow(r)) {
            const size_t er = (size_t)r * N + col;
            acc += (T)(1.0 - bc.alpha) * (x[(size_t)g0 * per + er] + x[(size_t)(g0 + 1) * per + er]);
          }
          const bool outflow = wall == 0 ? vx < 0 : vx > 0;
          if (mu == 0 && outflow) acc += (T)(lflux[wall] * h * h * 2.0 * fabs(vx));
        }
      }
    }
    out[mu * cs + idx] = acc;
  }
}

// ------------------------------------------------------------------ Heun stages
// Transpose of the two Heun stages with F(w) = C[w] + 2 (B x w_vec), given
// cg = C'(x)^T lam_F at the stage's state x:
//   stage 2 (x = w1):  out = lam_b / 2 + dt/2 (cg + 2 lam_b_vec x B),  gB += dt/2 * 2 sum_v x_vec x lam_b_vec
//   stage 1 (x = w):   out = lam_b / 2 + lam_1 + dt (cg + 2 lam_1_vec x B), gB += dt * 2 sum_v x_vec x lam_1_vec
// One workgroup per cell; gB (float64 [Nx][3]) accumulates.
template <typename T>
__global__ void k_heun_vjp(const T* __restrict__ lb, const T* __restrict__ l1, const T* __restrict__ cg,
                           const T* __restrict__ x, const double* __restrict__ B, T* __restrict__ out,
                           double* __restrict__ gB, T dt, int Nx, int N, int stage) {
  const int cell = blockIdx.x;
  const int per = N * N;
  const size_t cs = (size_t)Nx * per;
  const T B1 = B ? (T)B[3 * cell] : (T)0, B2 = B ? (T)B[3 * cell + 1] : (T)0, B3 = B ? (T)B[3 * cell + 2] : (T)0;
  const T* lf = stage == 2 ? lb : l1;
  const T coef = stage == 2 ? (T)0.5 * dt : dt;
  double s1 = 0, s2 = 0, s3 = 0;
  for (int e = threadIdx.x; e < per; e += blockDim.x) {
    const size_t o = (size_t)cell * per + e;
    const T a1 = lf[cs + o], a2 = lf[2 * cs + o], a3 = lf[3 * cs + o];
    const T m[4] = {(T)0, (T)2 * (a2 * B3 - a3 * B2), (T)2 * (a3 * B1 - a1 * B3), (T)2 * (a1 * B2 - a2 * B1)};
    for (int mu = 0; mu < 4; ++mu) {
      const size_t q = mu * cs + o;
      T v = (T)0.5 * lb[q] + coef * (cg[q] + m[mu]);
      if (stage == 1) v += l1[q];
      out[q] = v;
    }
    const T x1 = x[cs + o], x2 = x[2 * cs + o], x3 = x[3 * cs + o];
    s1 += (double)(x2 * a3 - x3 * a2);
    s2 += (double)(x3 * a1 - x1 * a3);
    s3 += (double)(x1 * a2 - x2 * a1);
  }
  __shared__ double red[3][256];
  red[0][threadIdx.x] = s1;
  red[1][threadIdx.x] = s2;
  red[2][threadIdx.x] = s3;
  __syncthreads();
  for (int o = blockDim.x / 2; o > 0; o >>= 1) {
    if (threadIdx.x < o)
      for (int k = 0; k < 3; ++k) red[k][threadIdx.x] += red[k][threadIdx.x + o];
    __syncthreads();
  }
  if (gB && threadIdx.x < 3) gB[3 * cell + threadIdx.x] += 2.0 * (double)coef * red[threadIdx.x][0];
}

}  // namespace qb
