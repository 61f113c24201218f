// Register-resident 2D FFT engine for gfx950 (wave64).
//
// A P x P complex field is spread over NT = P * TPR threads of a workgroup,
// TPR = P / E threads per line, E elements per thread.  Thread t owns line
// l = t / TPR and lane-in-line q (the TPR lanes of a line are adjacent lanes
// of one wavefront).  For TPR <= 4, q = t % TPR.  For TPR = 8 the lanes of
// the upper half are relabelled, q = p ^ 3 for p = t % 8 >= 4 (lanes
// 4, 5, 6, 7 hold q = 7, 6, 5, 4), so that the distance-4 partner of every
// lane, q ^ 4, is the lane 7 - p: one row_half_mirror move instead of a quad
// permute and a mirror.  The partners at distance 2 and 1 stay p ^ 2, p ^ 1.
//
//   "strided"  layout: element index  x = q + TPR * n,        n = 0..E-1
//   "blocked"  layout: element index  k + E * bitrev(q),      k = 0..E-1
//
// A forward line transform takes strided data to blocked spectra: an E-point
// FFT in registers on the stride-TPR subsequence, a twiddle w_P^{q k}, then a
// TPR-point DFT across the lanes (radix-2 decimation in frequency through
// lane shuffles, which leaves the output blocks in bit-reversed lane order).
// The inverse line transform runs the same steps backwards.  Both are
// unnormalized: inv(fwd(x)) = P x.
//
// 2D: rows (index x, line = y) and columns (index y, line = kx).  The field
// moves between row and column ownership through an LDS transpose, one real
// component at a time (both at once in workgroups that fill a CU and have
// the LDS for two planes), through a padded P x P buffer per component.
//
//   row real (strided in x) --fwd rows--> row spectra (blocked in kx)
//     --T1--> column real (strided in y) --fwd cols--> column spectra
//   and back with the inverse transforms and T2.
#pragma once
#include <hip/hip_runtime.h>

#include <utility>

namespace qb {

// ------------------------------------------------------------------ constexpr trig
// Taylor series after reduction to [-pi/4, pi/4]; used only for the compile-time
// twiddles of the in-register transforms.
constexpr double kPi = 3.14159265358979323846264338327950288;

constexpr double cx_sin_small(double x) {
  double term = x, sum = x;
  for (int k = 1; k < 14; ++k) {
    term *= -x * x / ((2.0 * k) * (2.0 * k + 1.0));
    sum += term;
  }
  return sum;
}
constexpr double cx_cos_small(double x) {
  double term = 1.0, sum = 1.0;
  for (int k = 1; k < 14; ++k) {
    term *= -x * x / ((2.0 * k - 1.0) * (2.0 * k));
    sum += term;
  }
  return sum;
}
// cos / sin of 2 pi a / b for integers 0 <= a < b, b a power of two.
constexpr double cx_cos_frac(int a, int b) {
  // octant reduction: angle = 2 pi a / b = (pi/4) * (8a/b)
  const int a8 = a * 8;
  const int oct = a8 / b;               // 0..7
  const double r = (double)(a8 - oct * b) / b * (kPi / 4.0);  // [0, pi/4)
  switch (oct) {
    case 0: return cx_cos_small(r);
    case 1: return cx_sin_small(kPi / 4.0 - r);
    case 2: return -cx_sin_small(r);
    case 3: return -cx_cos_small(kPi / 4.0 - r);
    case 4: return -cx_cos_small(r);
    case 5: return -cx_sin_small(kPi / 4.0 - r);
    case 6: return cx_sin_small(r);
    default: return cx_cos_small(kPi / 4.0 - r);
  }
}
constexpr double cx_sin_frac(int a, int b) {
  const int a8 = a * 8;
  const int oct = a8 / b;
  const double r = (double)(a8 - oct * b) / b * (kPi / 4.0);
  switch (oct) {
    case 0: return cx_sin_small(r);
    case 1: return cx_cos_small(kPi / 4.0 - r);
    case 2: return cx_cos_small(r);
    case 3: return cx_sin_small(kPi / 4.0 - r);
    case 4: return -cx_sin_small(r);
    case 5: return -cx_cos_small(kPi / 4.0 - r);
    case 6: return -cx_cos_small(r);
    default: return -cx_sin_small(kPi / 4.0 - r);
  }
}

template <int A, int B>
struct Tw {
  static constexpr double c = cx_cos_frac(A, B);
  static constexpr double s = cx_sin_frac(A, B);
};

constexpr int ilog2(int n) { return n <= 1 ? 0 : 1 + ilog2(n / 2); }
constexpr int bitrev_c(int v, int bits) {
  int r = 0;
  for (int i = 0; i < bits; ++i) r |= ((v >> i) & 1) << (bits - 1 - i);
  return r;
}
__host__ __device__ inline int bitrev_rt(int v, int bits) {
  int r = 0;
  for (int i = 0; i < bits; ++i) r |= ((v >> i) & 1) << (bits - 1 - i);
  return r;
}

// ------------------------------------------------------------------ in-register FFT
// y[k] = sum_n x[O + S n] exp(DIR * 2 pi i n k / E), natural order in and out.
template <typename T, int E, int DIR>
struct RegFft {
  template <int S, int O, int IN_N>
  static __device__ __forceinline__ void run(const T (&xr)[IN_N], const T (&xi)[IN_N], T (&yr)[E],
                                             T (&yi)[E]) {
    if constexpr (E == 1) {
      yr[0] = xr[O];
      yi[0] = xi[O];
    } else {
      constexpr int H = E / 2;
      T er[H], ei[H], orr[H], oi[H];
      RegFft<T, H, DIR>::template run<2 * S, O, IN_N>(xr, xi, er, ei);
      RegFft<T, H, DIR>::template run<2 * S, O + S, IN_N>(xr, xi, orr, oi);
      butterflies(er, ei, orr, oi, yr, yi, std::make_integer_sequence<int, H>{});
    }
  }

  template <int H, int... K>
  static __device__ __forceinline__ void butterflies(const T (&er)[H], const T (&ei)[H], const T (&orr)[H],
                                                     const T (&oi)[H], T (&yr)[E], T (&yi)[E],
                                                     std::integer_sequence<int, K...>) {
    (bfly<H, K>(er, ei, orr, oi, yr, yi), ...);
  }

  template <int H, int K>
  static __device__ __forceinline__ void bfly(const T (&er)[H], const T (&ei)[H], const T (&orr)[H],
                                              const T (&oi)[H], T (&yr)[E], T (&yi)[E]) {
    T tr, ti;
    if constexpr (K == 0) {
      tr = orr[K];
      ti = oi[K];
    } else if constexpr (4 * K == E) {
      // w = exp(DIR * i pi / 2) = DIR * i
      if constexpr (DIR < 0) {
        tr = oi[K];
        ti = -orr[K];
      } else {
        tr = -oi[K];
        ti = orr[K];
      }
    } else {
      constexpr T c = (T)Tw<K, E>::c;
      constexpr T s = (T)(DIR * Tw<K, E>::s);
      tr = orr[K] * c - oi[K] * s;
      ti = orr[K] * s + oi[K] * c;
    }
    yr[K] = er[K] + tr;
    yi[K] = ei[K] + ti;
    yr[K + H] = er[K] - tr;
    yi[K + H] = ei[K] - ti;
  }
};

template <typename T, int E, int DIR>
__device__ __forceinline__ void reg_fft(T (&zr)[E], T (&zi)[E]) {
  T yr[E], yi[E];
  RegFft<T, E, DIR>::template run<1, 0, E>(zr, zi, yr, yi);
#pragma unroll
  for (int k = 0; k < E; ++k) {
    zr[k] = yr[k];
    zi[k] = yi[k];
  }
}

// ------------------------------------------------------------------ lane shuffles
// Value of lane (lane ^ MASK) for MASK in {1, 2}, by a DPP quad_perm move,
// and for MASK = 7 the value of lane 7 - i in each group of 8 lanes
// (row_half_mirror): the distance-4 partner under the TPR = 8 lane labels.
template <int MASK>
__device__ __forceinline__ int xor_lane_i32(int v) {
  if constexpr (MASK == 1) {
    return __builtin_amdgcn_mov_dpp(v, 0xB1, 0xF, 0xF, false);  // quad_perm [1,0,3,2]
  } else if constexpr (MASK == 2) {
    return __builtin_amdgcn_mov_dpp(v, 0x4E, 0xF, 0xF, false);  // quad_perm [2,3,0,1]
  } else {
    static_assert(MASK == 7, "lane mask must be 1, 2 or 7");
    return __builtin_amdgcn_mov_dpp(v, 0x141, 0xF, 0xF, false);  // row_half_mirror
  }
}

template <int MASK>
__device__ __forceinline__ float xor_lane(float v) {
  return __int_as_float(xor_lane_i32<MASK>(__float_as_int(v)));
}

template <int MASK>
__device__ __forceinline__ double xor_lane(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = xor_lane_i32<MASK>((int)(b & 0xffffffffll));
  const int hi = xor_lane_i32<MASK>((int)(b >> 32));
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// ------------------------------------------------------------------ engine
template <typename T, int P_, int E_, bool XB_ = false>
struct Fft2 {
  static constexpr int P = P_;
  static constexpr int E = E_;
  static constexpr int TPR = P / E;
  static constexpr int NT = P * TPR;
  static constexpr int LB = ilog2(TPR);
  // LDS transpose layout: row kx holds y at y + off(kx), rows LD apart, with
  // off(kx) = (BW / TPR) * (kx / E), BW the number of elements per 128-byte
  // bank cycle, LD = P + BW + TPR.  Every transpose access of a wavefront then
  // falls into distinct banks, and each thread's E accesses differ by
  // compile-time constants (one address register per direction).
  static constexpr int BW = 128 / (int)sizeof(T);
  static constexpr int LD = P + BW + TPR;
  // The transposes can go through LDS in ROUNDS passes of P / ROUNDS kx rows
  // each (a smaller buffer, at the price of extra barriers and registers);
  // one pass unless QB_XPOSE_SPLIT_BYTES asks for a split.
#ifndef QB_XPOSE_SPLIT_BYTES
#define QB_XPOSE_SPLIT_BYTES (1 << 30)
#endif
  static constexpr int ROUNDS = (P * LD * (int)sizeof(T) > QB_XPOSE_SPLIT_BYTES && P / 2 >= E) ? 2 : 1;
  static constexpr int RP = P / ROUNDS;
  static constexpr int PLANE = RP * LD;  // one real plane of the transpose buffer
  // Kernels whose workgroups of 512 threads or more fill a compute unit on
  // their own (one per CU at their register use) may ask (XB_) to move the
  // real and imaginary planes together through two buffers: two barriers
  // per transpose instead of four, where every barrier idles the whole CU.
  static constexpr bool XB = XB_ && ROUNDS == 1 && NT >= 512 && 2 * PLANE * (int)sizeof(T) <= 96 * 1024;
  static constexpr int LDS_SCALARS = (XB ? 2 : 1) * PLANE;
  static_assert(TPR >= 1 && TPR <= 8 && (TPR & (TPR - 1)) == 0, "TPR must be 1, 2, 4 or 8");
  static_assert(E * TPR == P, "E * TPR must equal P");
  static_assert(P % BW == 0, "P must be a multiple of the bank width");

  int t, line, q, bq;
  T* lds;          // transpose buffer, LDS_SCALARS scalars
  const T* tw;     // LDS: (cos, sin)(2 pi q k / P) at [q][k], q < TPR, k < E, row stride TWS
  // padded row stride of the twiddle table: the TPR rows start in different banks
  static constexpr int TWS = 2 * E + 2;
  static constexpr int TW_SCALARS = TPR * TWS;

  // logical lane q of physical lane p (an involution, see the header)
  static __host__ __device__ constexpr int lane_label(int p) { return TPR == 8 ? p ^ (3 * (p >> 2)) : p; }

  __device__ __forceinline__ void init(T* lds_buf, const T* twi) {
    t = threadIdx.x;
    line = t / TPR;
    q = lane_label(t % TPR);
    bq = bitrev_rt(q, LB);
    lds = lds_buf;
    tw = twi;
  }
  __device__ __forceinline__ int sx(int n) const { return q + TPR * n; }     // strided index
  __device__ __forceinline__ int bk(int k) const { return k + E * bq; }      // blocked index
  // LDS position of (kx row inside the buffer, y) without the bank offset
  __device__ __forceinline__ int addr(int kxl, int y) const { return kxl * LD + y; }
  // bank offset of a kx row: spreads the TPR row groups kx / E over the banks
  __device__ __forceinline__ int off_of(int kx) const { return (BW / TPR) * (kx / E); }

  // w_P^{q k} multiply, sign SG (-1 forward, +1 inverse), k = 1..E-1
  template <int SG>
  __device__ __forceinline__ void twiddle(T (&zr)[E], T (&zi)[E]) const {
    // The table is constant, so the compiler would keep all E twiddles in
    // registers across the whole kernel; an opaque base index makes it load
    // them where they are used instead.
    int base = q * TWS;
    __asm__ volatile("" : "+v"(base));
#pragma unroll
    for (int k = 1; k < E; ++k) {
      const T* w = tw + base + 2 * k;
      const T c = w[0], s = SG < 0 ? -w[1] : w[1];
      const T r = zr[k] * c - zi[k] * s;
      zi[k] = zr[k] * s + zi[k] * c;
      zr[k] = r;
    }
  }

  // twiddle w_8^r, r = 0..3, of the H = 4 lane stage (conjugated for the
  // inverse), as (re, im)
  template <int SG>
  __device__ __forceinline__ void w8(int r, T& wr, T& wi) const {
    const T c = (T)0.70710678118654752440;
    wr = r == 0 ? (T)1 : (r == 1 ? c : (r == 2 ? (T)0 : -c));
    const T s = r == 0 ? (T)0 : (r == 2 ? (T)1 : c);
    wi = SG < 0 ? -s : s;
  }

  // Cross-lane DFT of size TPR for every k.  Forward (decimation in
  // frequency, natural lane order in, bit-reversed out):
  //   stage H = TPR/2 .. 1: lower lane z + o, upper lane (o - z) w_{2H}^{q mod H}
  // The H = 2 stage twiddle is w_4 = -i (lanes with q mod 4 = 3), applied as a
  // component swap; the H = 4 stage (TPR = 8) multiplies the upper lanes by
  // w_8^{q mod 4}.
  __device__ __forceinline__ void lanes_fwd(T (&zr)[E], T (&zi)[E]) const {
    if constexpr (TPR == 8) {
      const T sg = (q & 4) ? (T)-1 : (T)1;
      T wr, wi;
      w8<-1>((q & 4) ? (q & 3) : 0, wr, wi);
#pragma unroll
      for (int k = 0; k < E; ++k) {
        const T orr = xor_lane<7>(zr[k]), oi = xor_lane<7>(zi[k]);
        const T dr = sg * zr[k] + orr, di = sg * zi[k] + oi;
        zr[k] = dr * wr - di * wi;
        zi[k] = dr * wi + di * wr;
      }
    }
    if constexpr (TPR >= 4) {
      const T sg = (q & 2) ? (T)-1 : (T)1;
      const bool rot = (q & 3) == 3;
#pragma unroll
      for (int k = 0; k < E; ++k) {
        const T orr = xor_lane<2>(zr[k]), oi = xor_lane<2>(zi[k]);
        const T dr = sg * zr[k] + orr, di = sg * zi[k] + oi;
        zr[k] = rot ? di : dr;       // (d) * (-i) = (d_i, -d_r)
        zi[k] = rot ? -dr : di;
      }
    }
    if constexpr (TPR >= 2) {
      const T sg = (q & 1) ? (T)-1 : (T)1;
#pragma unroll
      for (int k = 0; k < E; ++k) {
        const T orr = xor_lane<1>(zr[k]), oi = xor_lane<1>(zi[k]);
        zr[k] = sg * zr[k] + orr;
        zi[k] = sg * zi[k] + oi;
      }
    }
  }
  // exact reverse of lanes_fwd (unnormalized: times TPR)
  __device__ __forceinline__ void lanes_inv(T (&zr)[E], T (&zi)[E]) const {
    if constexpr (TPR >= 2) {
      const T sg = (q & 1) ? (T)-1 : (T)1;
#pragma unroll
      for (int k = 0; k < E; ++k) {
        const T orr = xor_lane<1>(zr[k]), oi = xor_lane<1>(zi[k]);
        zr[k] = sg * zr[k] + orr;
        zi[k] = sg * zi[k] + oi;
      }
    }
    if constexpr (TPR >= 4) {
      const T sg = (q & 2) ? (T)-1 : (T)1;
      const bool rot = (q & 3) == 3;
#pragma unroll
      for (int k = 0; k < E; ++k) {
        // undo the -i of lanes q mod 4 = 3: multiply by +i = (-z_i, z_r)
        const T ar = rot ? -zi[k] : zr[k];
        const T ai = rot ? zr[k] : zi[k];
        const T orr = xor_lane<2>(ar), oi = xor_lane<2>(ai);
        zr[k] = sg * ar + orr;
        zi[k] = sg * ai + oi;
      }
    }
    if constexpr (TPR == 8) {
      const T sg = (q & 4) ? (T)-1 : (T)1;
      T wr, wi;
      w8<+1>((q & 4) ? (q & 3) : 0, wr, wi);
#pragma unroll
      for (int k = 0; k < E; ++k) {
        const T ar = zr[k] * wr - zi[k] * wi, ai = zr[k] * wi + zi[k] * wr;
        const T orr = xor_lane<7>(ar), oi = xor_lane<7>(ai);
        zr[k] = sg * ar + orr;
        zi[k] = sg * ai + oi;
      }
    }
  }

  // forward: strided -> blocked, exp(-2 pi i ...)
  __device__ __forceinline__ void fwd_line(T (&zr)[E], T (&zi)[E]) const {
    reg_fft<T, E, -1>(zr, zi);
    if constexpr (TPR > 1) {
      twiddle<-1>(zr, zi);
      lanes_fwd(zr, zi);
    }
  }

  // inverse: blocked -> strided, exp(+2 pi i ...), unnormalized
  __device__ __forceinline__ void inv_line(T (&zr)[E], T (&zi)[E]) const {
    if constexpr (TPR > 1) {
      lanes_inv(zr, zi);
      twiddle<+1>(zr, zi);
    }
    reg_fft<T, E, +1>(zr, zi);
  }

  // T1: row spectra (blocked in kx, line = y) -> column real (strided in y, line = kx)
  __device__ __forceinline__ void t_rows_to_cols(T (&zr)[E], T (&zi)[E]) const {
    if constexpr (XB) {
#pragma unroll
      for (int k = 0; k < E; ++k) {
        const int a = addr(bk(k), line) + off_of(bk(k));
        lds[a] = zr[k];
        lds[PLANE + a] = zi[k];
      }
      __syncthreads();
#pragma unroll
      for (int n = 0; n < E; ++n) {
        const int a = addr(line, sx(n)) + off_of(line);
        zr[n] = lds[a];
        zi[n] = lds[PLANE + a];
      }
      __syncthreads();
    } else {
      xpose_rb_to_cs(zr);
      xpose_rb_to_cs(zi);
    }
  }
  // T2: column real (strided in y, line = kx) -> row spectra (blocked in kx, line = y)
  __device__ __forceinline__ void t_cols_to_rows(T (&zr)[E], T (&zi)[E]) const {
    if constexpr (XB) {
#pragma unroll
      for (int n = 0; n < E; ++n) {
        const int a = addr(line, sx(n)) + off_of(line);
        lds[a] = zr[n];
        lds[PLANE + a] = zi[n];
      }
      __syncthreads();
#pragma unroll
      for (int k = 0; k < E; ++k) {
        const int a = addr(bk(k), line) + off_of(bk(k));
        zr[k] = lds[a];
        zi[k] = lds[PLANE + a];
      }
      __syncthreads();
    } else {
      xpose_cs_to_rb(zr);
      xpose_cs_to_rb(zi);
    }
  }

  // With ROUNDS > 1 a thread may receive its column elements in an earlier
  // round than the one in which it hands over its row elements, so received
  // values go to a separate array until every round is done.
  __device__ __forceinline__ void xpose_rb_to_cs(T (&z)[E]) const {
    if constexpr (ROUNDS == 1) {
#pragma unroll
      for (int k = 0; k < E; ++k) lds[addr(bk(k), line) + off_of(bk(k))] = z[k];
      __syncthreads();
#pragma unroll
      for (int n = 0; n < E; ++n) z[n] = lds[addr(line, sx(n)) + off_of(line)];
      __syncthreads();
    } else {
      T zn[E];
#pragma unroll
      for (int r = 0; r < ROUNDS; ++r) {
        if ((E * bq) / RP == r) {
#pragma unroll
          for (int k = 0; k < E; ++k) lds[addr(bk(k) - r * RP, line) + off_of(bk(k))] = z[k];
        }
        __syncthreads();
        if (line / RP == r) {
#pragma unroll
          for (int n = 0; n < E; ++n) zn[n] = lds[addr(line - r * RP, sx(n)) + off_of(line)];
        }
        __syncthreads();
      }
#pragma unroll
      for (int n = 0; n < E; ++n) z[n] = zn[n];
    }
  }
  __device__ __forceinline__ void xpose_cs_to_rb(T (&z)[E]) const {
    if constexpr (ROUNDS == 1) {
#pragma unroll
      for (int n = 0; n < E; ++n) lds[addr(line, sx(n)) + off_of(line)] = z[n];
      __syncthreads();
#pragma unroll
      for (int k = 0; k < E; ++k) z[k] = lds[addr(bk(k), line) + off_of(bk(k))];
      __syncthreads();
    } else {
      T zn[E];
#pragma unroll
      for (int r = 0; r < ROUNDS; ++r) {
        if (line / RP == r) {
#pragma unroll
          for (int n = 0; n < E; ++n) lds[addr(line - r * RP, sx(n)) + off_of(line)] = z[n];
        }
        __syncthreads();
        if ((E * bq) / RP == r) {
#pragma unroll
          for (int k = 0; k < E; ++k) zn[k] = lds[addr(bk(k) - r * RP, line) + off_of(bk(k))];
        }
        __syncthreads();
      }
#pragma unroll
      for (int k = 0; k < E; ++k) z[k] = zn[k];
    }
  }

  // full 2D: row real -> column spectra
  __device__ __forceinline__ void fwd2(T (&zr)[E], T (&zi)[E]) const {
    fwd_line(zr, zi);
    t_rows_to_cols(zr, zi);
    fwd_line(zr, zi);
  }
  // full 2D: column spectra -> row real
  __device__ __forceinline__ void inv2(T (&zr)[E], T (&zi)[E]) const {
    inv_line(zr, zi);
    t_cols_to_rows(zr, zi);
    inv_line(zr, zi);
  }
};

}  // namespace qb
