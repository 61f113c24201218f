// Device kernels of the spectral collision operator, transport and time step.
//
// Internal layouts (all per cell):
//   state     w[mu][cell][i][j], mu = 0..3 Pauli components (Sec. 3.1), on the
//             velocity grid v = (2L/N)(i - N/2, j - N/2).
//   P grid    the 2N x 2N zero-padded grid (Sec. 3.2), stored in FFT order:
//             real-space index x = p mod P for p in [-N, N-1] (spacing L/N, the
//             velocity grid sits on the even points), frequency index k = b mod P.
//   row real  real-space field, "strided" engine layout: element (x, y) lives
//             in thread t = y*TPR + x%TPR, slot n = x/TPR, stored at n*NT + t.
//   col spec  spectrum, "blocked" layout: element (kx, ky) lives in thread
//             t = kx*TPR + bitrev(ky/E), slot k = ky%E, stored at k*NT + t
//             (real and imaginary planes separately).
#pragma once
#include "qb_fft.hpp"

namespace qb {

template <typename T, int P>
struct Cfg;
template <>
struct Cfg<double, 32> { static constexpr int E = 16; };
template <>
struct Cfg<double, 64> { static constexpr int E = 16; };
template <>
struct Cfg<double, 128> { static constexpr int E = 16; };
template <>
struct Cfg<float, 32> { static constexpr int E = 16; };
template <>
struct Cfg<float, 64> { static constexpr int E = 16; };
template <>
struct Cfg<float, 128> { static constexpr int E = 16; };

// Device-side view of the plan's tables and buffers (all device pointers).
template <typename T>
struct DevPlan {
  int Nx, N, J, M, P;
  T L;
  T wc, wd;  // weights of C_c and C_d in the assembled C (term selection; 1, 1 for the full operator)
  // tables, col-spec layout [J][P*P] unless noted
  const T* tw;     // [P][2] (cos, sin)(2 pi i / P)
  const T* phip;   // phi_R(b . theta'_j)                       (I_1 inner)
  const T* Kt;     // sum_j omega_G[j][j'] phi_R(b . theta_j) / P^2 (I_1 outer)
  const T* psi;    // psi_R(b . theta_j)                        (I_2)
  const T* psip;   // psi_R(b . theta_j^perp)                   (I_2, I_4 inner)
  const T* psiw;   // (pi/J) psi_R(b . theta_j) / P^2           (I_4 outer)
  const T* psips;  // psi_R(b . theta_j^perp) / P^2             (I_3 multiplier)
  const unsigned* negk;  // [P*P] col spec position of -k for the position of k
  const T* phx;    // [J][M][P][2] exp(i pi rho_m theta_j,x b_x / L)
  const T* phy;    // [J][M][P][2] exp(i pi rho_m theta_j,y b_y / L)
  const T* wm;     // [M] (pi/J) w_m
  // work buffers
  T* spec;   // [cells][4][2][P*P]  w_hat_mu, col spec
  T* wP;     // [cells][5][P*P]     w_mu and f0 = 2 w0 - 1 on the P grid, row real
  T* terms;  // [cells][11][P*P]    I_1 (3), I_4 (4), I_2 (one per Pauli component) real-space fields
  T* acc;    // [cells][7][2][P*P]  spectral accumulators of the I_1 / I_4 tasks
  T* i3s;    // [cells][J][4 or 6][P*P]  shifted fields of the current (j, m) (+ partner sums)
  T* i3o;    // [cells][J][4][P*P]  I_3 partial sums over m, per j
  T* i3sum;  // [cells][4][P*P]     assembled real-space fields of C
  T* i3p;    // [cells][J][4][P*P]  partner-node spectra of I_3 per j (2 packed pairs, re/im, col spec)
  T* i3ps;   // [cells][4][P*P]     i3p summed over j
  // adjoint work buffers (present once the plan's adjoint is enabled)
  T* lamP;   // [cells][4][P*P]     cotangent of the assembled fields, row real
  T* acot;   // [cells][16][P*P]    assembly cotangents: g (3), y (4), S (1), b (4), w direct (4)
  T* gspec;  // [cells][11][2][P*P] cotangents of w_hat from I_1 (3), I_4 (4), I_2 (4), col spec
  T* gf0;    // [cells][7][P*P]     f0 cotangents of the I_1 / I_4 tasks, row real
  T* i3g;    // [cells][J][8][P*P]  I_3 adjoint per (cell, j): w cotangent (4, row real),
             //                     packed w_hat cotangents (2 pairs x re/im, col spec)
  T* i3sb;   // [cells][J][4][P*P]  cotangent of the shifted fields of the current (j, m)
  T* i3t;    // [cells][J][4][P*P]  shifted cotangents of the I_3 sums for the current (j, m)
  T* lamh;   // [cells][4][P*P]     spectrum of lamP, packed pairs, col spec
  T* gsum;   // [cells][8][P*P]     gathered cotangents (k_grad_pre)
  T* fwa;    // [cells][7][2][P*P]  spectral accumulators of the forward I_1 / I_4 fields in k_terms_vjp
};

// ------------------------------------------------------------------ helpers
template <int P>
__device__ __forceinline__ int centered(int k) {
  return k < P / 2 ? k : k - P;
}

template <typename T>
__device__ __forceinline__ void cmul(T ar, T ai, T br, T bi, T& cr, T& ci) {
  cr = ar * br - ai * bi;
  ci = ar * bi + ai * br;
}

// Raw buffer access: one 128-bit resource per array (scalar registers), a
// per-thread byte offset in one vector register and a uniform byte offset,
// so the E loads of a thread need no per-element address registers.
using rsrc_t = __amdgpu_buffer_rsrc_t;
template <typename T>
__device__ __forceinline__ rsrc_t mkbuf(const T* p, size_t n) {
  return __builtin_amdgcn_make_buffer_rsrc((void*)p, 0, (int)(n * sizeof(T)), 0x00020000);
}
template <typename T>
__device__ __forceinline__ T bld(rsrc_t r, unsigned voff, unsigned soff) {
  if constexpr (sizeof(T) == 4) {
    return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, 0));
  } else {
    return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0));
  }
}
template <typename T>
__device__ __forceinline__ void bst(rsrc_t r, T v, unsigned voff, unsigned soff) {
  if constexpr (sizeof(T) == 4) {
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), r, voff, soff, 0);
  } else {
    typedef unsigned u2 __attribute__((ext_vector_type(2)));
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u2, v), r, voff, soff, 0);
  }
}

// Buffer-to-LDS copy of one float field in the engine's element order:
// element n of thread t (byte n NT 4 + 4 t past soff) lands in lds[n NT + t].
// Each load writes the 64 lanes of a wavefront to 64 consecutive LDS words
// starting at a wave-uniform address, so a thread later reads only words
// its own wavefront wrote: the wait below, not a barrier, orders them.
template <typename T, int NT, int E>
__device__ __forceinline__ void fetch_lds(rsrc_t r, T* lds, unsigned voff, unsigned soff) {
  static_assert(sizeof(T) == 4, "buffer-to-LDS loads of 4-byte elements");
  typedef __attribute__((address_space(3))) void* lds_ptr;
  const unsigned wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  unsigned lb = (unsigned)(size_t)(__attribute__((address_space(3))) T*)lds + 256u * wave;
  unsigned sb = soff;
  // opaque here, so the per-element scalar offsets below are formed at the
  // loads instead of being hoisted out of the caller's loops (which would
  // hold 2 E scalar registers for the whole kernel)
  __asm__ volatile("" : "+s"(lb), "+s"(sb));
#pragma unroll
  for (int n = 0; n < E; ++n)
    __builtin_amdgcn_raw_ptr_buffer_load_lds(r, (lds_ptr)(size_t)(lb + n * NT * 4), 4, voff, sb + n * NT * 4, 0, 0);
}
// The same for elements of any size: dword d of every element lands in LDS
// plane d (NT E dwords each), read back with lds_elem.
template <typename T, int NT, int E>
__device__ __forceinline__ void fetch_lds_dw(rsrc_t r, unsigned* lds, unsigned voff, unsigned soff) {
  typedef __attribute__((address_space(3))) void* lds_ptr;
  constexpr int DW = (int)sizeof(T) / 4;
  const unsigned wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  unsigned lb = (unsigned)(size_t)(__attribute__((address_space(3))) unsigned*)lds + 256u * wave;
  unsigned sb = soff;
  __asm__ volatile("" : "+s"(lb), "+s"(sb));
#pragma unroll
  for (int dw = 0; dw < DW; ++dw)
#pragma unroll
    for (int n = 0; n < E; ++n)
      __builtin_amdgcn_raw_ptr_buffer_load_lds(r, (lds_ptr)(size_t)(lb + (dw * NT * E + n * NT) * 4), 4,
                                               voff + 4 * dw, sb + n * NT * (int)sizeof(T), 0, 0);
}
template <typename T, int NT, int E>
__device__ __forceinline__ T lds_elem(const unsigned* lds, int n, unsigned t) {
  if constexpr (sizeof(T) == 4) {
    return __builtin_bit_cast(T, lds[n * NT + t]);
  } else {
    const unsigned long long lo = lds[n * NT + t], hi = lds[NT * E + n * NT + t];
    return __builtin_bit_cast(T, lo | (hi << 32));
  }
}
// Wait until every buffer load of this wavefront (the LDS copies included)
// has completed; returns the thread index through the wait so that LDS
// reads addressed with it cannot move above the wait.
__device__ __forceinline__ unsigned lds_fetch_wait() {
  unsigned t = threadIdx.x;
  __asm__ volatile("s_waitcnt vmcnt(0)" : "+v"(t));
  return t;
}

// XCD-aware block order: consecutive logical tasks share an XCD (its L2).
__device__ __forceinline__ int xcd_task(int b, int nb) {
  if ((nb & 7) != 0) return b;
  return (b & 7) * (nb >> 3) + (b >> 3);
}

// Velocity-grid row index of the padded-grid point x = q + TPR n (FFT order),
// for even x: i = centered(x)/2 + N/2.  For even q the wrap at x = N falls at
// n = N / TPR whatever q is, so the offset is affine in n with a
// compile-time break.
template <int P, int TPR>
__device__ __forceinline__ int vel_index(int q, int n) {
  constexpr int N = P / 2;
  return q / 2 + (TPR / 2) * n + N / 2 - (n >= N / TPR ? N : 0);
}

// ------------------------------------------------------------------ layout kernels
// API complex [cells][N][N][2][2] -> Pauli state w[4][cells][N][N]
template <typename T, typename TA>
__global__ void k_api_to_state(const TA* __restrict__ W, T* __restrict__ w, int ncells, int N, int Nx) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  const int per = N * N;
  if (idx >= ncells * per) return;
  const TA* m = W + (size_t)idx * 8;  // W00 W01 W10 W11, each (re, im)
  const TA w00r = m[0], w01r = m[2], w01i = m[3], w10r = m[4], w10i = m[5], w11r = m[6];
  const size_t cs = (size_t)Nx * per;
  w[idx] = (T)(0.5 * ((double)w00r + (double)w11r));
  w[cs + idx] = (T)(0.5 * ((double)w10r + (double)w01r));
  w[2 * cs + idx] = (T)(0.5 * ((double)w10i - (double)w01i));
  w[3 * cs + idx] = (T)(0.5 * ((double)w00r - (double)w11r));
}

// Pauli state -> API complex
template <typename T, typename TA>
__global__ void k_state_to_api(const T* __restrict__ w, TA* __restrict__ W, int ncells, int N, int Nx) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  const int per = N * N;
  if (idx >= ncells * per) return;
  const size_t cs = (size_t)Nx * per;
  const T a0 = w[idx], a1 = w[cs + idx], a2 = w[2 * cs + idx], a3 = w[3 * cs + idx];
  TA* m = W + (size_t)idx * 8;
  m[0] = (TA)(a0 + a3);
  m[1] = (TA)0;
  m[2] = (TA)a1;
  m[3] = (TA)(-a2);
  m[4] = (TA)a1;
  m[5] = (TA)a2;
  m[6] = (TA)(a0 - a3);
  m[7] = (TA)0;
}

// ------------------------------------------------------------------ engine setup
template <typename T, int P, int E, bool XB = false>
struct Kern {
  using Eng = Fft2<T, P, E, XB>;
  static constexpr int NT = Eng::NT;
  static constexpr int TPR = Eng::TPR;
  static constexpr int FSZ = P * P;
  static constexpr int LDS = Eng::LDS_SCALARS + Eng::TW_SCALARS;
  // occupancy target of the transform kernels (waves per SIMD): two
  // workgroups per compute unit where the field is small enough
#ifndef QB_F32_P128_WAVES
#define QB_F32_P128_WAVES 1
#endif
  static constexpr int WAVES = (sizeof(T) == 4 && P == 128) ? QB_F32_P128_WAVES : 1;
};

template <typename T, int P, int E, bool XB>
__device__ __forceinline__ void setup(Fft2<T, P, E, XB>& eng, T* smem, const T* tw) {
  using F = Fft2<T, P, E, XB>;
  T* t2 = smem + F::LDS_SCALARS;
  // tw holds [q][k] rows of 2E scalars; LDS rows are TWS apart
  for (int i = threadIdx.x; i < 2 * P; i += blockDim.x) t2[(i / (2 * E)) * F::TWS + i % (2 * E)] = tw[i];
  __syncthreads();
  eng.init(smem, t2);
}

// ------------------------------------------------------------------ dft_in
// w_mu(v_n) -> w_hat_mu on Xi (Nyquist zeroed, padded to P, col spec), and the
// trigonometric interpolants w_mu, f0 = 2 w0 - 1 on the P grid (row real).
template <typename T, int P, int E>
__global__ __launch_bounds__((Fft2<T, P, E>::NT)) void k_dft_in(DevPlan<T> d, const T* __restrict__ w, int cell0) {
  using K = Kern<T, P, E>;
  constexpr unsigned S = sizeof(T);
  __shared__ T smem[K::LDS];
  Fft2<T, P, E> eng;
  setup(eng, smem, d.tw);
  const int cell = cell0 + blockIdx.x;
  const int N = P / 2;
  const unsigned vo = threadIdx.x * S;
  const size_t cs = (size_t)d.Nx * N * N;
  const int y = eng.line;
  const rsrc_t rs = mkbuf(d.spec + (size_t)blockIdx.x * 8 * K::FSZ, 8 * K::FSZ);
  const rsrc_t rw = mkbuf(d.wP + (size_t)blockIdx.x * 5 * K::FSZ, 5 * K::FSZ);
  const T inv_n2 = (T)1 / (T)(N * N);
  const int bx = centered<P>(eng.line);
  const bool kx_in = bx > -N / 2 && bx < N / 2;
#pragma unroll 1
  for (int mu = 0; mu < 4; ++mu) {
    T zr[E], zi[E];
    // the velocity grid sits on the even points of the padded grid
    const bool on_grid = ((eng.q | y) & 1) == 0;
    const T* wrow = w + mu * cs + (size_t)cell * N * N + (centered<P>(y) / 2 + N / 2);
#pragma unroll
    for (int n = 0; n < E; ++n) {
      zr[n] = on_grid ? wrow[vel_index<P, K::TPR>(eng.q, n) * N] : (T)0;
      zi[n] = 0;
    }
    eng.fwd2(zr, zi);
#pragma unroll
    for (int k = 0; k < E; ++k) {
      const int by = centered<P>(eng.bk(k));
      const bool in = kx_in && by > -N / 2 && by < N / 2;
      bst<T>(rs, in ? zr[k] * inv_n2 : (T)0, vo, ((2 * mu) * K::FSZ + k * K::NT) * S);
      bst<T>(rs, in ? zi[k] * inv_n2 : (T)0, vo, ((2 * mu + 1) * K::FSZ + k * K::NT) * S);
    }
  }
#pragma unroll 1
  for (int pr = 0; pr < 2; ++pr) {
    T zr[E], zi[E];
    const unsigned fa = 2 * (2 * pr) * K::FSZ, fb = 2 * (2 * pr + 1) * K::FSZ;
#pragma unroll
    for (int k = 0; k < E; ++k) {
      const unsigned o = k * K::NT;
      // (a_r + i a_i) + i (b_r + i b_i)
      zr[k] = bld<T>(rs, vo, (fa + o) * S) - bld<T>(rs, vo, (fb + K::FSZ + o) * S);
      zi[k] = bld<T>(rs, vo, (fa + K::FSZ + o) * S) + bld<T>(rs, vo, (fb + o) * S);
    }
    eng.inv2(zr, zi);
#pragma unroll
    for (int n = 0; n < E; ++n) {
      const unsigned o = n * K::NT;
      bst<T>(rw, zr[n], vo, ((2 * pr) * K::FSZ + o) * S);
      bst<T>(rw, zi[n], vo, ((2 * pr + 1) * K::FSZ + o) * S);
      if (pr == 0) bst<T>(rw, (T)2 * zr[n] - (T)1, vo, (4 * K::FSZ + o) * S);
    }
  }
}

// ------------------------------------------------------------------ I_1, I_4, I_2
// task 0..2: I_1[f0, w_l, .] (l = task + 1), hoisted outer kernel K_j'
// task 3..6: I_4[f0, w_g, .] (g = task - 3)
// Both: sum_j outer_j(p) FFT( f0 * IFFT(inner_j w_hat_g) ), then one IFFT.
// task 7..10: I_2 accumulator S = sum_mu S_mu, one Pauli component
//            mu = task - 7 per task: S_mu = sum_j (pi/J) eta_mu
//            IFFT(psi_j w_hat_mu) IFFT(psi'_j w_hat_mu)   (real space)
constexpr int kTermPlanes = 11;
template <typename T, int P, int E>
__global__ __launch_bounds__((Fft2<T, P, E>::NT)) void k_terms(DevPlan<T> d, int ncells) {
  using K = Kern<T, P, E>;
  constexpr unsigned S = sizeof(T);
  __shared__ T smem[K::LDS];
  Fft2<T, P, E> eng;
  setup(eng, smem, d.tw);
  // one (cell, task) per workgroup, or grid-stride when persistent
#pragma unroll 1
  for (int pt = blockIdx.x; pt < ncells * kTermPlanes; pt += gridDim.x) {
  const int cell = pt / kTermPlanes;
  const int task = pt % kTermPlanes;
  const unsigned vo = threadIdx.x * S;
  const rsrc_t rs = mkbuf(d.spec + (size_t)cell * 8 * K::FSZ, 8 * K::FSZ);
  const rsrc_t rw = mkbuf(d.wP + (size_t)cell * 5 * K::FSZ, 5 * K::FSZ);
  const rsrc_t ro = mkbuf(d.terms + ((size_t)cell * kTermPlanes + task) * K::FSZ, K::FSZ);
  const size_t tabn = (size_t)d.J * K::FSZ;
  if (task < 7) {
    const int g = task < 3 ? task + 1 : task - 3;
    const rsrc_t rin = mkbuf(task < 3 ? d.phip : d.psip, tabn);
    const rsrc_t rout = mkbuf(task < 3 ? d.Kt : d.psiw, tabn);
    const rsrc_t ra = mkbuf(d.acc + ((size_t)cell * 7 + task) * 2 * K::FSZ, 2 * K::FSZ);
    const unsigned fg = 2 * g * K::FSZ;
    // in_j, out_j are real with one parity in k (odd for I_1, even for
    // I_4) and w_hat_g is the spectrum of a real field, so a_j is real up
    // to a fixed phase: directions j, j+1 share both transforms, with
    // coefficients (i_j + i i_j+1, o_j - i o_j+1) for even tables and
    // (i_j+1 - i i_j, o_j+1 + i o_j) for odd ones.  The real part of the
    // final inverse transform is the field; the cross terms the sharing
    // adds are imaginary there.
    const bool odd = task < 3;
#pragma unroll 1
    for (int j = 0; j < d.J; j += 2) {
      T zr[E], zi[E];
      const unsigned t1 = j * K::FSZ, t2 = t1 + K::FSZ;
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
        const T f = bld<T>(rw, vo, (4 * K::FSZ + n * K::NT) * S);
        zr[n] *= f;
        zi[n] *= f;
      }
      eng.fwd2(zr, zi);
#pragma unroll
      for (int k = 0; k < E; ++k) {
        const unsigned o = k * K::NT;
        const T o1 = bld<T>(rout, vo, (t1 + o) * S), o2 = bld<T>(rout, vo, (t2 + o) * S);
        const T cr = odd ? o2 : o1, ci = odd ? o1 : -o2;
        T ar = cr * zr[k] - ci * zi[k], ai = cr * zi[k] + ci * zr[k];
        // read at j = 0 too (not yet written) and dropped by a select
        const T pr = bld<T>(ra, vo, o * S), pi = bld<T>(ra, vo, (K::FSZ + o) * S);
        ar += j != 0 ? pr : (T)0;
        ai += j != 0 ? pi : (T)0;
        bst<T>(ra, ar, vo, o * S);
        bst<T>(ra, ai, vo, (K::FSZ + o) * S);
      }
    }
    T zr[E], zi[E];
#pragma unroll
    for (int k = 0; k < E; ++k) {
      const unsigned o = k * K::NT;
      zr[k] = bld<T>(ra, vo, o * S);
      zi[k] = bld<T>(ra, vo, (K::FSZ + o) * S);
    }
    eng.inv2(zr, zi);
#pragma unroll
    for (int n = 0; n < E; ++n) bst<T>(ro, zr[n], vo, (n * K::NT) * S);
  } else {
    // one Pauli component per task: S_mu = sum_j e_mu A_j,mu B_j,mu
    const int mu = task - 7;
    const unsigned fm = 2 * mu * K::FSZ;
    const T e = (T)(kPi / d.J) * (mu == 0 ? (T)1 : (T)-1);
    T Sacc[E];
#pragma unroll
    for (int n = 0; n < E; ++n) Sacc[n] = 0;
    const rsrc_t rps = mkbuf(d.psi, tabn);
    const rsrc_t rpp = mkbuf(d.psip, tabn);
#pragma unroll 1
    for (int j = 0; j < d.J; ++j) {
      const unsigned tj = j * K::FSZ;
      T zr[E], zi[E];
#pragma unroll
      for (int k = 0; k < E; ++k) {
        const unsigned o = k * K::NT;
        const T ar = bld<T>(rs, vo, (fm + o) * S), ai = bld<T>(rs, vo, (fm + K::FSZ + o) * S);
        const T a = bld<T>(rps, vo, (tj + o) * S), b = bld<T>(rpp, vo, (tj + o) * S);
        // w_hat psi + i w_hat psi'
        zr[k] = ar * a - ai * b;
        zi[k] = ai * a + ar * b;
      }
      eng.inv2(zr, zi);
#pragma unroll
      for (int n = 0; n < E; ++n) Sacc[n] += e * zr[n] * zi[n];
    }
#pragma unroll
    for (int n = 0; n < E; ++n) bst<T>(ro, Sacc[n], vo, (n * K::NT) * S);
  }
  }  // tasks
}

// ------------------------------------------------------------------ I_3
// One workgroup per (cell, j); loops over the Gauss-Legendre nodes in
// symmetric pairs (m, m' = M-1-m), rho_m' = -rho_m, w_m' = w_m (the middle
// node of an odd M runs alone).  With s_nu = S w_nu the field shifted by
// node m (S = inv2(exp(i alpha_jm . b) fwd2(.)) / P^2) and the packed
// convolutions Phi_a,b = Psi(w_a s_b), Psi = inv2(psi'_j / P^2 fwd2(.)):
//   node m :  o_b  += c sum_a eta_a s_a Phi_a,b                 (real space)
//   node m':  o'_a  = c S^{-1} sum_b eta_b w_b Phi_a,b
// because translations commute with Psi and distribute over products whose
// band stays inside the padded grid; the aliased part of the last product
// falls outside Xi, which the output keeps.  o' is accumulated as a
// spectrum, conj(phase) fwd2(sign_a o'_a) with the sign of the B term
// (-1 for a = 0), packed (0 + i1), (2 + i3), into i3p[cell][j].
// c = (pi/J) w_m.  Per pair: 2 shift transforms, 8 packed convolutions of 2
// transforms each, 2 transforms of the partner sums.
// Register plan.  One workgroup of NT threads puts NT / 256 waves on each
// SIMD (at least one), so a thread may hold 512 / that many VGPRs (at most
// 256).  The working field takes 2 E values; the partner sums of a row pair
// 2 E more (PAIR: in registers where they fit, otherwise in two planes of
// the shifted-field buffer); the four shifted fields 4 E more (SREG:
// otherwise they go through a per-workgroup buffer).  About 48 VGPRs go to
// addresses and temporaries.  (The thresholds were checked against the
// compiler's register reports for every compiled tile.)  The kernel is
// compiled with and without node pairing; pairing is the default on every
// tile and wins on each.
template <typename T, int P, int E>
struct I3Regs {
  static constexpr int NT = P * (P / E);
  static constexpr int WPS = NT / 256 > 1 ? NT / 256 : 1;
  static constexpr int BUDGET = 512 / WPS < 256 ? 512 / WPS : 256;
  static constexpr int F = E * (int)sizeof(T) / 4;  // VGPRs of one field
  static constexpr bool PAIR = 2 * F + 2 * F + 48 <= BUDGET;
  // the transforms need about 2 E more values of temporaries once the
  // shifted fields live in registers too
  template <bool PR>
  static constexpr bool sreg() {
    return 2 * F + (PR ? 2 * F : 0) + 4 * F + 2 * F + 48 <= BUDGET;
  }
  // one float32 field of LDS beside the transpose buffer, where it fits in
  // the 160 KB of a compute unit and one workgroup fills the compute unit
  // anyway (P = 128): the staging buffer of the accumulator prefetches
  template <bool PR, int LDS_SCALARS>
  static constexpr bool lds_field() {
    return PR && !sreg<PR>() && P == 128 && sizeof(T) == 4 &&
           (LDS_SCALARS + P * P) * (int)sizeof(T) <= 160 * 1024;
  }
  // At P = 64 with E = 16 (256 threads) the register plan leaves two
  // workgroups per compute unit, each with half of the 160 KB of LDS: the
  // output accumulators that fit beside the transpose buffer stay in LDS for
  // the whole node loop (3 in float32, 1 in float64) instead of going
  // through memory at every node.
  template <bool PR, int LDS_SCALARS>
  static constexpr int lds_acc() {
    if (!PR || P != 64 || NT != 256) return 0;
    const int k = (80 * 1024 - LDS_SCALARS * (int)sizeof(T)) / (P * P * (int)sizeof(T));
    return k < 0 ? 0 : (k > 4 ? 4 : k);
  }
};

// Planes per (cell, j) of the shifted-field buffer i3s: the four shifted
// fields, and in float64 two more for partner sums that do not fit in
// registers.
template <typename T>
constexpr int kI3sPlanes = sizeof(T) == 8 ? 6 : 4;

template <typename T>
__device__ __forceinline__ T pick4(int i, T a, T b, T c, T d) {
  return i == 0 ? a : (i == 1 ? b : (i == 2 ? c : d));
}

template <typename T, int P, int E, bool PAIR>
__global__ __launch_bounds__((Fft2<T, P, E>::NT)) __attribute__((amdgpu_waves_per_eu(Kern<T, P, E>::WAVES))) void k_i3(DevPlan<T> d, int ncells) {
  using K = Kern<T, P, E, true>;
  constexpr unsigned S = sizeof(T);
  constexpr bool SREG = I3Regs<T, P, E>::template sreg<PAIR>();
  // Paired nodes keep the partner sums of a row pair in registers where the
  // register plan allows (PREG); otherwise (float64 at P = 128, and the
  // 32-element float64 tile at P = 64) they accumulate in two more planes
  // of the shifted-field buffer (PMEM) instead of spilling.
  constexpr bool PREG = PAIR && I3Regs<T, P, E>::PAIR;
  constexpr bool PMEM = PAIR && !PREG;
  static_assert(!(PMEM && SREG), "partner sums in memory need the shifted-field buffer");
  // the current row pair's two shifted fields in registers for the nu loop
  // (saves two field reads per convolution), with at most 16 registers per
  // field: it fits the unpaired kernel; in the paired float32 kernel at
  // P = 128 it pushes about 38 registers to scratch and still runs 4 %
  // faster, the field reads it saves waiting right after a transform
  constexpr bool AREG = !SREG && I3Regs<T, P, E>::F <= 16;
  // PF: the accumulator field read back after a convolution is fetched
  // into LDS (buffer-to-LDS loads, no registers) before the convolution
  // starts, so its latency hides behind the transforms
  constexpr bool PF = I3Regs<T, P, E>::template lds_field<PAIR, K::LDS>();
  __shared__ T smem[K::LDS];
  __shared__ T pf[PF ? K::FSZ : 1];
  // KRES accumulator fields resident in LDS; each thread touches only its
  // own elements, so no barrier guards them
  constexpr int KRES = I3Regs<T, P, E>::template lds_acc<PAIR, K::LDS>();
  __shared__ T acc[KRES > 0 ? KRES * K::FSZ : 1];
  // elements between scheduling barriers in the element loops, which bound
  // the loads in flight (measured: 4 at P = 128, 8 at P = 64)
  constexpr int SG = P >= 128 ? 4 : 8;
  const unsigned tid = threadIdx.x;
  typename K::Eng eng;
  setup(eng, smem, d.tw);
  // one (cell, j) task per workgroup, or grid-stride over the tasks when
  // the launch is persistent (a grid that is a multiple of 8 keeps every
  // cell's tasks on the XCD that runs them)
  const int ntask = ncells * d.J;
#pragma unroll 1
  for (int pt = blockIdx.x; pt < ntask; pt += gridDim.x) {
  const int task = xcd_task(pt, ntask);
  const int cell = task / d.J;
  const int j = task % d.J;
  const unsigned vo = threadIdx.x * S;
  const size_t tb = (size_t)cell * d.J + j;
  const rsrc_t rs = mkbuf(d.spec + (size_t)cell * 8 * K::FSZ, 8 * K::FSZ);
  const rsrc_t rw = mkbuf(d.wP + (size_t)cell * 5 * K::FSZ, 5 * K::FSZ);
  const rsrc_t ro = mkbuf(d.i3o + tb * 4 * K::FSZ, 4 * K::FSZ);
  const rsrc_t rp = mkbuf(d.i3p + tb * 4 * K::FSZ, 4 * K::FSZ);
  const rsrc_t rb = mkbuf(SREG ? d.i3o : d.i3s + tb * kI3sPlanes<T> * K::FSZ, kI3sPlanes<T> * K::FSZ);
  const rsrc_t rm = mkbuf(d.psips + (size_t)j * K::FSZ, K::FSZ);
  const int kx = eng.line;
  T s[SREG ? 4 : 1][SREG ? E : 1];
  const int nnode = PAIR ? (d.M + 1) / 2 : d.M;
#pragma unroll 1
  for (int m = 0; m < nnode; ++m) {
    const bool paired = PAIR && m != d.M - 1 - m;
    const T* px = d.phx + (((size_t)j * d.M + m) * P) * 2;
    const T* py = d.phy + (((size_t)j * d.M + m) * P) * 2 + 2 * E * eng.bq;
    const T pxr = px[2 * kx], pxi = px[2 * kx + 1];
    // shifted fields
#pragma unroll
    for (int pr = 0; pr < 2; ++pr) {
      const unsigned fa = 2 * (2 * pr) * K::FSZ, fb = 2 * (2 * pr + 1) * K::FSZ;
      T zr[E], zi[E];
#pragma unroll
      for (int k = 0; k < E; ++k) {
        const unsigned o = k * K::NT;
        T er, ei;
        cmul(pxr, pxi, py[2 * k], py[2 * k + 1], er, ei);
        T ar, ai, br, bi;
        cmul(bld<T>(rs, vo, (fa + o) * S), bld<T>(rs, vo, (fa + K::FSZ + o) * S), er, ei, ar, ai);
        cmul(bld<T>(rs, vo, (fb + o) * S), bld<T>(rs, vo, (fb + K::FSZ + o) * S), er, ei, br, bi);
        zr[k] = ar - bi;
        zi[k] = ai + br;
        if (k % SG == SG - 1) __builtin_amdgcn_sched_barrier(0);
      }
      eng.inv2(zr, zi);
#pragma unroll
      for (int n = 0; n < E; ++n) {
        if constexpr (SREG) {
          s[SREG ? 2 * pr : 0][n] = zr[n];
          s[SREG ? 2 * pr + 1 : 0][n] = zi[n];
        } else {
          bst<T>(rb, zr[n], vo, ((2 * pr) * K::FSZ + n * K::NT) * S);
          bst<T>(rb, zi[n], vo, ((2 * pr + 1) * K::FSZ + n * K::NT) * S);
        }
      }
    }
    const T wgt = d.wm[m];
#pragma unroll 1
    for (int mp = 0; mp < 2; ++mp) {
      const int m0 = 2 * mp, m1 = 2 * mp + 1;
      // partner sums of this pair of rows a = m0, m1 (sign of the B term folded in)
      // (in registers; with PMEM in planes 4, 5 of the shifted-field buffer)
      T pa[PREG ? E : 1], pb[PREG ? E : 1];
      if constexpr (PREG) {
#pragma unroll
        for (int n = 0; n < E; ++n) pa[n] = pb[n] = 0;
      }
      const T sa_sign = m0 == 0 ? (T)-1 : (T)1;
      // the row pair's shifted fields, in registers for the nu loop
      T ra[AREG ? E : 1], rbv[AREG ? E : 1];
      if constexpr (AREG) {
#pragma unroll
        for (int n = 0; n < E; ++n) {
          ra[AREG ? n : 0] = bld<T>(rb, vo, (m0 * K::FSZ + n * K::NT) * S);
          rbv[AREG ? n : 0] = bld<T>(rb, vo, (m1 * K::FSZ + n * K::NT) * S);
        }
      }
      const bool first = m == 0 && mp == 0;
#pragma unroll 1
      for (int nu = 0; nu < 4; ++nu) {
        // (fetched on the first pass too, where the values go unused: a
        // branch here would split the block the scheduler works on)
        if constexpr (PF) fetch_lds<T, K::NT, E>(ro, pf, vo, nu * K::FSZ * S);
        T zr[E], zi[E];
#pragma unroll
        for (int n = 0; n < E; ++n) {
          const unsigned o = n * K::NT;
          T sv;
          if constexpr (SREG)
            sv = pick4(nu, s[0][n], s[SREG ? 1 : 0][n], s[SREG ? 2 : 0][n], s[SREG ? 3 : 0][n]);
          else
            sv = bld<T>(rb, vo, (nu * K::FSZ + o) * S);
          zr[n] = bld<T>(rw, vo, (m0 * K::FSZ + o) * S) * sv;
          zi[n] = bld<T>(rw, vo, (m1 * K::FSZ + o) * S) * sv;
          if (n % SG == SG - 1) __builtin_amdgcn_sched_barrier(0);
        }
        eng.fwd2(zr, zi);
#pragma unroll
        for (int k = 0; k < E; ++k) {
          const T a = bld<T>(rm, vo, (k * K::NT) * S);
          zr[k] *= a;
          zi[k] *= a;
          if (k % SG == SG - 1) __builtin_amdgcn_sched_barrier(0);
        }
        eng.inv2(zr, zi);
        const T e0 = m0 == 0 ? wgt : -wgt;
        // c eta_nu, zero for the middle node of an odd M (no partner): the
        // partner sums then take zeros instead of a branch per element
        const T ew = !paired ? (T)0 : (nu == 0 ? wgt : -wgt);
        const unsigned pt = PF ? lds_fetch_wait() : 0u;
        const bool res = KRES > 0 && nu < KRES;
        T* const al = acc + (KRES > 0 && res ? nu * K::FSZ : 0) + tid;
#pragma unroll
        for (int n = 0; n < E; ++n) {
          const unsigned o = n * K::NT;
          T sa, sb;
          if constexpr (SREG) {
            sa = mp == 0 ? s[0][n] : s[SREG ? 2 : 0][n];
            sb = mp == 0 ? s[SREG ? 1 : 0][n] : s[SREG ? 3 : 0][n];
          } else if constexpr (AREG) {
            sa = ra[AREG ? n : 0];
            sb = rbv[AREG ? n : 0];
          } else {
            sa = bld<T>(rb, vo, (m0 * K::FSZ + o) * S);
            sb = bld<T>(rb, vo, (m1 * K::FSZ + o) * S);
          }
          const unsigned off = (nu * K::FSZ + o) * S;
          T v = e0 * sa * zr[n] - wgt * sb * zi[n];
          // the accumulator is read on the first pass too (in bounds, not
          // yet written) and the value dropped by a select: uniform branches
          // here would cut the element loop into separately scheduled blocks
          if (KRES > 0 && res) {
            const T prev = al[KRES > 0 ? o : 0];
            v += first ? (T)0 : prev;
            al[KRES > 0 ? o : 0] = v;
          } else {
            const T prev = PF ? pf[PF ? o + pt : 0] : bld<T>(ro, vo, off);
            v += first ? (T)0 : prev;
            bst<T>(ro, v, vo, off);
          }
          if constexpr (PREG) {
            const T wv = ew * bld<T>(rw, vo, (nu * K::FSZ + o) * S);
            pa[PREG ? n : 0] += sa_sign * wv * zr[n];
            pb[PREG ? n : 0] += wv * zi[n];
          } else if constexpr (PMEM) {
            // first nu of the row pair: the old value is dropped by a select
            const T wv = ew * bld<T>(rw, vo, (nu * K::FSZ + o) * S);
            const unsigned qa = (4 * K::FSZ + o) * S, qb = (5 * K::FSZ + o) * S;
            const T pva = bld<T>(rb, vo, qa), pvb = bld<T>(rb, vo, qb);
            bst<T>(rb, sa_sign * wv * zr[n] + (nu != 0 ? pva : (T)0), vo, qa);
            bst<T>(rb, wv * zi[n] + (nu != 0 ? pvb : (T)0), vo, qb);
          }
          if (n % SG == SG - 1) __builtin_amdgcn_sched_barrier(0);
        }
      }
      // spectrum of the partner sums: conj(phase) fwd2(pa + i pb), accumulated.
      // Only its entries on Xi reach the output (k_combine keeps Xi), so
      // the other lanes' buffer accesses get an offset past the buffer:
      // their loads return 0 and their stores are dropped, without memory
      // traffic and without a branch.
      const unsigned fr = (2 * mp) * K::FSZ, fi = (2 * mp + 1) * K::FSZ;
      const int bx = centered<P>(kx);
      const bool kx_in = bx > -P / 4 && bx < P / 4;
      auto xi_off = [&](int k) {
        const int by = centered<P>(eng.bk(k));
        return (kx_in && by > -P / 4 && by < P / 4) ? vo : 0x80000000u;
      };
      if (paired) {
        T zr[E], zi[E];
#pragma unroll
        for (int n = 0; n < E; ++n) {
          if constexpr (PMEM) {
            zr[n] = bld<T>(rb, vo, (4 * K::FSZ + n * K::NT) * S);
            zi[n] = bld<T>(rb, vo, (5 * K::FSZ + n * K::NT) * S);
          } else {
            zr[n] = pa[PREG ? n : 0];
            zi[n] = pb[PREG ? n : 0];
          }
        }
        eng.fwd2(zr, zi);
#pragma unroll
        for (int k = 0; k < E; ++k) {
          const unsigned o = k * K::NT;
          const unsigned vk = xi_off(k);
          T er, ei;
          cmul(pxr, pxi, py[2 * k], py[2 * k + 1], er, ei);
          T xr, xi;
          cmul(zr[k], zi[k], er, -ei, xr, xi);
          const T pr0 = bld<T>(rp, vk, (fr + o) * S);
          const T pi0 = bld<T>(rp, vk, (fi + o) * S);
          xr += m != 0 ? pr0 : (T)0;
          xi += m != 0 ? pi0 : (T)0;
          bst<T>(rp, xr, vk, (fr + o) * S);
          bst<T>(rp, xi, vk, (fi + o) * S);
          if (k % SG == SG - 1) __builtin_amdgcn_sched_barrier(0);
        }
      } else if (m == 0) {
        // no partner spectrum (unpaired kernel, or a single node)
#pragma unroll
        for (int k = 0; k < E; ++k) {
          const unsigned vk = xi_off(k);
          bst<T>(rp, (T)0, vk, (fr + k * K::NT) * S);
          bst<T>(rp, (T)0, vk, (fi + k * K::NT) * S);
        }
      }
    }
  }
  // the LDS-resident accumulators go to memory once
  if constexpr (KRES > 0) {
#pragma unroll 1
    for (int f = 0; f < KRES; ++f) {
#pragma unroll
      for (int n = 0; n < E; ++n) bst<T>(ro, acc[f * K::FSZ + n * K::NT + tid], vo, (f * K::FSZ + n * K::NT) * S);
    }
  }
  }  // tasks
}

// Real-space P-grid fields of C, elementwise: sums the per-j partials of I_3
// and assembles the Pauli components (C_c + pi (A + B + Cq), see k_combine)
// into i3sum[cell][mu]; sums the partner-node spectra of I_3 into i3ps on
// Xi (the only entries k_i3 writes and k_combine reads; 0 elsewhere).
template <typename T, int P, int E>
__global__ void k_assemble(DevPlan<T> d, int ncells) {
  using Eng = Fft2<T, P, E>;
  constexpr int fsz = P * P;
  const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (size_t)ncells * fsz) return;
  const size_t cell = idx / fsz, e = idx % fsz;
  const size_t per = (size_t)4 * fsz;
  // col spec position e = k NT + t: frequency (kx, ky) = (t / TPR, k + E bitrev(q))
  const int t = (int)(e % Eng::NT), kk = (int)(e / Eng::NT);
  const int bx = centered<P>(t / Eng::TPR);
  const int by = centered<P>(kk + E * bitrev_rt(Eng::lane_label(t % Eng::TPR), Eng::LB));
  const bool on_xi = bx > -P / 4 && bx < P / 4 && by > -P / 4 && by < P / 4;
  const T* o3 = d.i3o + cell * d.J * per + e;
  const T* p3 = d.i3p + cell * d.J * per + e;
  T b[4] = {0, 0, 0, 0}, q[4] = {0, 0, 0, 0};
  for (int j = 0; j < d.J; ++j)
    for (int nu = 0; nu < 4; ++nu) {
      b[nu] += o3[(size_t)j * per + (size_t)nu * fsz];
      if (on_xi) q[nu] += p3[(size_t)j * per + (size_t)nu * fsz];
    }
  T* ps = d.i3ps + cell * per + e;
  for (int nu = 0; nu < 4; ++nu) ps[(size_t)nu * fsz] = q[nu];
  const T* wp = d.wP + cell * 5 * fsz + e;
  const T* tr = d.terms + cell * kTermPlanes * fsz + e;
  const T w0 = wp[0], w1 = wp[fsz], w2 = wp[2 * fsz], w3 = wp[3 * fsz];
  const T g1 = tr[0], g2 = tr[fsz], g3 = tr[2 * fsz];
  const T y0 = tr[3 * fsz], y1 = tr[4 * fsz], y2 = tr[5 * fsz], y3 = tr[6 * fsz];
  const T Sv = (tr[7 * fsz] + tr[8 * fsz]) + (tr[9 * fsz] + tr[10 * fsz]);
  const T pi = (T)kPi, two = (T)2;
  T* r = d.i3sum + cell * per + e;
  // A: 2 <w3, w4>_eta (1 - W1); B: -2 <w3, w4>_eta (eta w2).sigma;
  // Cq: f0(v+u) {W1, (eta w2).sigma};  C_c,k = -2 eps_klm A^G_l w_m
  const T pd = d.wd * pi, wc = d.wc;
  r[0] = pd * (two * Sv * ((T)1 - w0) - two * b[0] + two * (y0 * w0 - y1 * w1 - y2 * w2 - y3 * w3));
  r[fsz] = -wc * two * (g2 * w3 - g3 * w2) + pd * (-two * Sv * w1 + two * b[1] + two * (y0 * w1 - y1 * w0));
  r[2 * fsz] = -wc * two * (g3 * w1 - g1 * w3) + pd * (-two * Sv * w2 + two * b[2] + two * (y0 * w2 - y2 * w0));
  r[3 * fsz] = -wc * two * (g1 * w2 - g2 * w1) + pd * (-two * Sv * w3 + two * b[3] + two * (y0 * w3 - y3 * w0));
}

// ------------------------------------------------------------------ combine
// Transform the assembled real-space P-grid fields of C (Pauli components,
// k_assemble), add the partner-node spectra of I_3 (times 2 pi, the B term
// with its sign already applied), keep Xi without its -N/2 rows and
// columns, and evaluate on the velocity grid:  c[mu][cell][i][j].
template <typename T, int P, int E>
__global__ __launch_bounds__((Fft2<T, P, E>::NT)) void k_combine(DevPlan<T> d, T* __restrict__ c, int cell0) {
  using K = Kern<T, P, E>;
  constexpr unsigned S = sizeof(T);
  __shared__ T smem[K::LDS];
  Fft2<T, P, E> eng;
  setup(eng, smem, d.tw);
  const int lc = blockIdx.x;
  const int cell = cell0 + lc;
  const int N = P / 2;
  const unsigned vo = threadIdx.x * S;
  const rsrc_t r3 = mkbuf(d.i3sum + (size_t)lc * 4 * K::FSZ, 4 * K::FSZ);
  const rsrc_t rps = mkbuf(d.i3ps + (size_t)lc * 4 * K::FSZ, 4 * K::FSZ);
  const size_t cs = (size_t)d.Nx * N * N;
#pragma unroll 1
  for (int pr = 0; pr < 2; ++pr) {
    T zr[E], zi[E];
#pragma unroll
    for (int n = 0; n < E; ++n) {
      const unsigned o = n * K::NT;
      zr[n] = bld<T>(r3, vo, ((2 * pr) * K::FSZ + o) * S);
      zi[n] = bld<T>(r3, vo, ((2 * pr + 1) * K::FSZ + o) * S);
    }
    eng.fwd2(zr, zi);
    const int bx = centered<P>(eng.line);
    const bool kx_in = bx > -N / 2 && bx < N / 2;
    const T sc = (T)1 / (T)(P * P);
    const T tp = d.wd * (T)(2.0 * kPi);  // B term of the partner nodes: pi * 2 * (sign folded in)
#pragma unroll
    for (int k = 0; k < E; ++k) {
      const unsigned o = k * K::NT;
      const int by = centered<P>(eng.bk(k));
      const bool in = kx_in && by > -N / 2 && by < N / 2;
      const T ar = bld<T>(rps, vo, ((2 * pr) * K::FSZ + o) * S), ai = bld<T>(rps, vo, ((2 * pr + 1) * K::FSZ + o) * S);
      zr[k] = in ? (zr[k] + tp * ar) * sc : (T)0;
      zi[k] = in ? (zi[k] + tp * ai) * sc : (T)0;
    }
    eng.inv2(zr, zi);
    const int y = eng.line;
    if (((eng.q | y) & 1) == 0) {
      T* ca = c + (2 * pr) * cs + (size_t)cell * N * N + (centered<P>(y) / 2 + N / 2);
      T* cb = ca + cs;
#pragma unroll
      for (int n = 0; n < E; ++n) {
        const int i = vel_index<P, K::TPR>(eng.q, n);
        ca[i * N] = zr[n];
        cb[i * N] = zi[n];
      }
    }
  }
}

// ------------------------------------------------------------------ Heun stage
// stage 1: w1 = w + dt (c + 2 B x w);  stage 2: w = (w + w1 + dt (c + 2 B x w1)) / 2
template <typename T>
__global__ void k_heun(T* __restrict__ w, T* __restrict__ w1, const T* __restrict__ c,
                       const double* __restrict__ B, T dt, int Nx, int N, int stage) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  const int per = N * N;
  if (idx >= Nx * per) return;
  const int cell = idx / per;
  const size_t cs = (size_t)Nx * per;
  const T* src = stage == 1 ? w : w1;
  const T a1 = src[cs + idx], a2 = src[2 * cs + idx], a3 = src[3 * cs + idx];
  T m1 = 0, m2 = 0, m3 = 0;
  if (B) {
    const T B1 = (T)B[3 * cell], B2 = (T)B[3 * cell + 1], B3 = (T)B[3 * cell + 2];
    m1 = (T)2 * (B2 * a3 - B3 * a2);
    m2 = (T)2 * (B3 * a1 - B1 * a3);
    m3 = (T)2 * (B1 * a2 - B2 * a1);
  }
  const T f[4] = {c[idx], c[cs + idx] + m1, c[2 * cs + idx] + m2, c[3 * cs + idx] + m3};
  for (int mu = 0; mu < 4; ++mu) {
    const size_t o = mu * cs + idx;
    if (stage == 1)
      w1[o] = w[o] + dt * f[mu];
    else
      w[o] = (T)0.5 * (w[o] + w1[o] + dt * f[mu]);
  }
}

// Exact flow of the field term over time tau: dw/dt = 2 B x w turns the
// Bloch vector of cell x about B(x) by the angle 2 |B| tau (Rodrigues'
// formula); w0 is unchanged.  State w[4][Nx][N][N].
template <typename T>
__global__ void k_rotate(T* __restrict__ w, const double* __restrict__ B, double tau, int Nx, int N) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  const int per = N * N;
  if (idx >= Nx * per) return;
  const int cell = idx / per;
  const size_t cs = (size_t)Nx * per;
  const double b1 = B[3 * cell], b2 = B[3 * cell + 1], b3 = B[3 * cell + 2];
  const double nb = sqrt(b1 * b1 + b2 * b2 + b3 * b3);
  if (!(nb > 0.0)) return;
  const double th = 2.0 * nb * tau;
  const T c = (T)cos(th), sn = (T)sin(th), k1 = (T)(b1 / nb), k2 = (T)(b2 / nb), k3 = (T)(b3 / nb);
  const T v1 = w[cs + idx], v2 = w[2 * cs + idx], v3 = w[3 * cs + idx];
  const T kv = (k1 * v1 + k2 * v2 + k3 * v3) * ((T)1 - c);
  w[cs + idx] = v1 * c + (k2 * v3 - k3 * v2) * sn + k1 * kv;
  w[2 * cs + idx] = v2 * c + (k3 * v1 - k1 * v3) * sn + k2 * kv;
  w[3 * cs + idx] = v3 * c + (k1 * v2 - k2 * v1) * sn + k3 * kv;
}

// ------------------------------------------------------------------ transport
struct BcDev {
  int kind;          // 0 periodic, 1 Dirichlet, 2 Maxwell
  double alpha;
  double Z;          // incoming flux of W_FD (Maxwell)
};

template <typename T>
__device__ __forceinline__ T minmod(T a, T b) {
  return (a * b > (T)0) ? (fabs(a) <= fabs(b) ? a : b) : (T)0;
}

// Slope of a cell from its one-sided differences a = W_{j+1} - W_j and
// b = W_j - W_{j-1} (Sec. 4: minmod, or another standard limiter):
// 0 minmod; 1 superbee, the larger of minmod(a, 2b) and minmod(2a, b);
// 2 monotonized central, minmod((a + b)/2, minmod(2a, 2b)); 3 van Leer,
// (a |b| + |a| b) / (|a| + |b|).
template <typename T>
__device__ __forceinline__ T slope(int kind, T a, T b) {
  switch (kind) {
    case 1: {
      const T s1 = minmod(a, (T)2 * b), s2 = minmod((T)2 * a, b);
      return fabs(s1) >= fabs(s2) ? s1 : s2;
    }
    case 2:
      return minmod((T)0.5 * (a + b), minmod((T)2 * a, (T)2 * b));
    case 3: {
      const T den = fabs(a) + fabs(b);
      return den > (T)0 ? (a * fabs(b) + fabs(a) * b) / den : (T)0;
    }
    default:
      return minmod(a, b);
  }
}

// Maxwell: outgoing number flux Fbar = h^2 sum_out tr W_b |v_x| of the cell
// next to each Maxwell wall (float64), one workgroup per wall.
template <typename T>
__global__ void k_maxwell_flux(const T* __restrict__ w, double* __restrict__ flux, int Nx, int N, double L,
                               int left_maxwell, int right_maxwell) {
  const int wall = blockIdx.x;  // 0 left, 1 right
  if ((wall == 0 && !left_maxwell) || (wall == 1 && !right_maxwell)) return;
  const int cell = wall == 0 ? 0 : Nx - 1;
  const double h = 2.0 * L / N;
  double s = 0.0;
  for (int e = threadIdx.x; e < N * N; e += blockDim.x) {
    const int i = e / N;
    const double vx = h * (i - N / 2);
    const bool out = wall == 0 ? vx < 0 : vx > 0;
    if (out) s += 2.0 * (double)w[((size_t)cell * N + i) * N + (e % N)] * fabs(vx);
  }
  __shared__ double red[256];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int o = blockDim.x / 2; o > 0; o >>= 1) {
    if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) flux[wall] = h * h * red[0];
}

// Value of the ghost-extended state at cell c (c < 0 or c >= Nx are ghost
// cells), component mu, velocity point e = i*N + j (Sec. 2 walls):
// periodic wrap; at a wall, the inflow state at incoming v_x (Dirichlet Phi,
// Maxwell (1 - alpha) W_b(-v_x, v_y) + alpha W_FD Fbar / Z), a copy of the
// adjacent cell otherwise; the row v_x = -L has no mirror and counts as
// outgoing at a Maxwell wall.
template <typename T>
__device__ __forceinline__ T ext_value(const T* __restrict__ w, const T* __restrict__ bcw,
                                       const double* __restrict__ flux, const BcDev& bl, const BcDev& br, int mu,
                                       int c, int e, int i, T vx, int Nx, int N, size_t cs) {
  const int per = N * N;
  if (c >= 0 && c < Nx) return w[mu * cs + (size_t)c * per + e];
  if (bl.kind == 0) {
    c = ((c % Nx) + Nx) % Nx;
    return w[mu * cs + (size_t)c * per + e];
  }
  const bool left = c < 0;
  const BcDev& bc = left ? bl : br;
  const int adj = left ? 0 : Nx - 1;
  const T* ws = bcw + (size_t)(left ? 0 : 1) * 4 * per + (size_t)mu * per;
  bool inflow = left ? (vx > (T)0) : (vx < (T)0);
  if (bc.kind == 2 && !left && i == 0) inflow = false;  // v_x = -L: no mirror
  if (!inflow) return w[mu * cs + (size_t)adj * per + e];
  if (bc.kind == 1) return ws[e];
  const int mi = N - i;  // mirrored v_x row
  const T wb = w[mu * cs + (size_t)adj * per + (size_t)mi * N + (e % N)];
  const double fz = flux[left ? 0 : 1] / bc.Z;
  return (T)(1.0 - bc.alpha) * wb + (T)(bc.alpha * fz) * ws[e];
}

// One step of eq. slopeLimiterStep of length dt, all cells and velocities.
// bcw: [2 walls][4][N][N] wall states (Dirichlet Phi or Maxwell W_FD).
// The Nx cells start at w / wn; components are Ntot * N * N apart (Ntot
// the cell count of the whole array, which may hold several problems).
template <typename T>
__global__ void k_transport(const T* __restrict__ w, T* __restrict__ wn, const T* __restrict__ bcw,
                            const double* __restrict__ flux, BcDev bl, BcDev br, T dt, int Nx, int N, T L,
                            int Ntot, int limiter) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  const int per = N * N;
  if (idx >= Nx * per) return;
  const int cell = idx / per;
  const int e = idx % per;
  const int i = e / N;
  const T h = (T)2 * L / (T)N;
  const T vx = h * (T)(i - N / 2);
  const T dx = (T)1 / (T)Nx;
  const size_t cs = (size_t)Ntot * per;
  T gval[4][5];
  for (int mu = 0; mu < 4; ++mu)
    for (int o = -2; o <= 2; ++o)
      gval[mu][o + 2] = ext_value(w, bcw, flux, bl, br, mu, cell + o, e, i, vx, Nx, N, cs);
  const T nu = dt * vx / dx;
  const T sg = vx > (T)0 ? (T)1 : (vx < (T)0 ? (T)-1 : (T)0);
  const T lim = (T)0.5 * (sg - nu);
  const T av = fabs(vx);
  for (int mu = 0; mu < 4; ++mu) {
    const T* g = gval[mu];
    const T Sm = slope(limiter, g[2] - g[1], g[1] - g[0]);
    const T S0 = slope(limiter, g[3] - g[2], g[2] - g[1]);
    const T Sp = slope(limiter, g[4] - g[3], g[3] - g[2]);
    const T upd = -vx * (g[3] - g[1]) + av * (g[3] - (T)2 * g[2] + g[1]) +
                  lim * (-vx * (Sp - Sm) + av * (Sp - (T)2 * S0 + Sm));
    wn[mu * cs + idx] = g[2] + dt / ((T)2 * dx) * upd;
  }
}

// ------------------------------------------------------------------ batch helpers
// dst[0..n) = src[0..n), or zeros for a NULL source (a problem without field)
static __global__ void k_copy_f64(const double* __restrict__ src, double* __restrict__ dst, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = src ? src[i] : 0.0;
}

// one problem's moments [snap][Nx][7] out of the batch moments [snap][Ntot][7]
static __global__ void k_scatter_moments(const double* __restrict__ src, double* __restrict__ dst, int nsnap, int Ntot,
                                  int off, int Nx) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int per = Nx * 7;
  if (i >= nsnap * per) return;
  const int snap = i / per, r = i % per;
  dst[i] = src[((size_t)snap * Ntot + off) * 7 + r];
}

// ------------------------------------------------------------------ moments
template <typename T>
__global__ void k_moments(const T* __restrict__ w, double* __restrict__ mom, int Nx, int N, double L) {
  const int cell = blockIdx.x;
  const int per = N * N;
  const size_t cs = (size_t)Nx * per;
  const double h = 2.0 * L / N;
  double acc[7] = {0, 0, 0, 0, 0, 0, 0};
  for (int e = threadIdx.x; e < per; e += blockDim.x) {
    const double vx = h * (e / N - N / 2), vy = h * (e % N - N / 2);
    const size_t o = (size_t)cell * per + e;
    const double a0 = (double)w[o];
    acc[0] += a0;
    acc[1] += (double)w[cs + o];
    acc[2] += (double)w[2 * cs + o];
    acc[3] += (double)w[3 * cs + o];
    acc[4] += vx * 2.0 * a0;
    acc[5] += vy * 2.0 * a0;
    acc[6] += 0.5 * (vx * vx + vy * vy) * 2.0 * a0;
  }
  __shared__ double red[7][256];
  for (int k = 0; k < 7; ++k) red[k][threadIdx.x] = acc[k];
  __syncthreads();
  for (int o = blockDim.x / 2; o > 0; o >>= 1) {
    if (threadIdx.x < o)
      for (int k = 0; k < 7; ++k) red[k][threadIdx.x] += red[k][threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x < 7) mom[(size_t)cell * 7 + threadIdx.x] = h * h * red[threadIdx.x][0];
}

}  // namespace qb
