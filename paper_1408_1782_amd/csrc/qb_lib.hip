// Host side of the solver: plan creation (quadrature tables of Sec. 3.2,
// device buffers), launch sequences of the step, batches, tuning and the C
// ABI declared in qb.h.  The collision pipelines (the FFT kernels of every
// tile shape) are compiled in the qb_tiles_*.hip units.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <algorithm>
#include <cstring>
#include <map>
#include <mutex>
#include <tuple>
#include <string>
#include <vector>

#include "qb_plan.hpp"
#include "qb_diag.hpp"

namespace {
thread_local std::string g_last_error;
}  // namespace

bool hip_ok(hipError_t e, const char* what) {
  if (e == hipSuccess) return true;
  g_last_error = std::string(what) + ": " + hipGetErrorString(e);
  return false;
}

void set_error(const char* what) { g_last_error = what; }

int persistent_grid(const void* kern, int threads) {
  static std::mutex mu;
  static std::map<std::pair<const void*, int>, int> cache;
  int dev = 0;
  (void)hipGetDevice(&dev);
  std::lock_guard<std::mutex> lock(mu);
  auto it = cache.find({kern, dev});
  if (it != cache.end()) return it->second;
  int per_cu = 0, cus = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, threads, 0) != hipSuccess) per_cu = 1;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) cus = 8;
  const int g = std::max(8, (std::max(per_cu, 1) * std::max(cus, 1)) / 8 * 8);
  cache[{kern, dev}] = g;
  return g;
}

namespace {

// ------------------------------------------------------------------ quadrature (host, float64)
// phi_R(x) = int_0^R sin(pi x r / L) dr = (2L/(pi x)) sin^2(pi R x / (2L)), phi_R(0) = 0
double phi_R(double x, double L, double R) {
  if (x == 0.0) return 0.0;
  const double s = std::sin(M_PI * R * x / (2.0 * L));
  return 2.0 * L / (M_PI * x) * s * s;
}
// psi_R(x) = int_{-R}^{R} exp(i pi x r / L) dr = (2L/(pi x)) sin(pi R x / L), psi_R(0) = 2R
double psi_R(double x, double L, double R) {
  if (x == 0.0) return 2.0 * R;
  return 2.0 * L / (M_PI * x) * std::sin(M_PI * R * x / L);
}

// Gauss-Legendre nodes / weights on [-1, 1] by Newton iteration on P_M.
void gauss_legendre(int M, std::vector<double>& x, std::vector<double>& w) {
  x.assign(M, 0.0);
  w.assign(M, 0.0);
  for (int i = 0; i < M; ++i) {
    double z = std::cos(M_PI * (i + 0.75) / (M + 0.5));
    double dp = 1.0;
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = z;
      for (int k = 2; k <= M; ++k) {
        const double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      double pm = M == 1 ? z : p1, pm1 = M == 1 ? 1.0 : p0;
      if (M == 1) {
        pm = z;
        pm1 = 1.0;
      }
      dp = M * (z * pm - pm1) / (z * z - 1.0);
      const double dz = pm / dp;
      z -= dz;
      if (std::fabs(dz) < 1e-16) break;
    }
    // recompute derivative at the converged node
    double p0 = 1.0, p1 = z;
    for (int k = 2; k <= M; ++k) {
      const double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
      p0 = p1;
      p1 = p2;
    }
    const double pm = M == 1 ? z : p1, pm1 = M == 1 ? 1.0 : p0;
    dp = M * (z * pm - pm1) / (z * z - 1.0);
    x[i] = -z;  // ascending order
    w[i] = 2.0 / ((1.0 - z * z) * dp * dp);
  }
}

// Tile shapes (elements per thread E; lanes per line P / E) compiled for
// each padded grid size; the first is the default, qb_plan_tune picks one.
std::vector<int> tile_candidates(int P) {
  switch (P) {
    case 32: return {16, 8};
    case 64: return {16, 32, 8};
    default: return {16, 32};
  }
}

int cfg_E(int precision, int P) {
  if (precision == QB_F64) return P == 32 ? qb::Cfg<double, 32>::E : (P == 64 ? qb::Cfg<double, 64>::E : qb::Cfg<double, 128>::E);
  return P == 32 ? qb::Cfg<float, 32>::E : (P == 64 ? qb::Cfg<float, 64>::E : qb::Cfg<float, 128>::E);
}

}  // namespace

namespace {

// copy a float64 host table, converted to T, into reserved device memory
template <typename T>
bool put(void* dst, const std::vector<double>& v) {
  std::vector<T> h(v.size());
  for (size_t i = 0; i < v.size(); ++i) h[i] = (T)v[i];
  return hip_ok(hipMemcpy(dst, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice), "hipMemcpy");
}

// col spec position of frequency indices (kx, ky) (FFT order): block ky / E
// sits in the lane whose logical label is its bit reversal (the engine's
// lane labels relabel the upper half of an 8-lane line, an involution)
inline size_t colspec_index(int kx, int ky, int E, int TPR, int NT) {
  const int lb = qb::ilog2(TPR);
  const int q = qb::bitrev_rt(ky / E, lb);
  const int lane = TPR == 8 ? q ^ (3 * (q >> 2)) : q;
  const int t = kx * TPR + lane;
  return (size_t)(ky % E) * NT + t;
}

inline int centered_h(int k, int P) { return k < P / 2 ? k : k - P; }

// Reserve the workspace of one tile shape's table set (twiddles, phi',
// K, psi, psi', weighted psi, psi' / P^2, the position of -k).
template <typename T>
bool reserve_layout_tables(qb_plan_s* pl, int E, qb_plan_s::TabSet& ts) {
  const size_t P = pl->P, J = pl->prob.J, FSZ = P * P, b = sizeof(T);
  ts.E = E;
  ts.built = false;
  return pl->alloc(&ts.tw, 2 * P * b) && pl->alloc(&ts.phip, J * FSZ * b) && pl->alloc(&ts.Kt, J * FSZ * b) &&
         pl->alloc(&ts.psi, J * FSZ * b) && pl->alloc(&ts.psip, J * FSZ * b) && pl->alloc(&ts.psiw, J * FSZ * b) &&
         pl->alloc(&ts.psips, J * FSZ * b) && pl->alloc(&ts.negk, FSZ * sizeof(unsigned));
}

// Compute the table set of tile shape ts.E in float64 and copy it into its
// reserved memory (Sec. 3.2: theta grids, phi_R, omega_G, psi_R).
template <typename T>
bool fill_layout_tables(qb_plan_s* pl, qb_plan_s::TabSet& ts) {
  const qb_problem& p = pl->prob;
  const int E = ts.E;
  const int P = pl->P, TPR = P / E, NT = P * TPR, J = p.J;
  const double L = p.L, R = p.R;
  const size_t FSZ = (size_t)P * P;
  // (cos, sin)(2 pi q k / P) at [q][k], q < TPR, k < E  (engine twiddles)
  std::vector<double> tw(2 * P);
  for (int q = 0; q < TPR; ++q)
    for (int k = 0; k < E; ++k) {
      const int i = q * E + k;
      tw[2 * i] = std::cos(2.0 * M_PI * ((q * k) % P) / P);
      tw[2 * i + 1] = std::sin(2.0 * M_PI * ((q * k) % P) / P);
    }
  std::vector<double> th_c(J), th_s(J), thp_c(J), thp_s(J);
  for (int j = 0; j < J; ++j) {
    th_c[j] = std::cos(j * M_PI / J);
    th_s[j] = std::sin(j * M_PI / J);
    thp_c[j] = std::cos((j + 0.5) * M_PI / J);
    thp_s[j] = std::sin((j + 0.5) * M_PI / J);
  }
  // omega_G[j][j'] = -(2 pi / J)^2 / (theta_j . theta'_j')   (eq. approxG)
  std::vector<double> wG((size_t)J * J);
  for (int j = 0; j < J; ++j)
    for (int jp = 0; jp < J; ++jp)
      wG[(size_t)j * J + jp] = -std::pow(2.0 * M_PI / J, 2) / (th_c[j] * thp_c[jp] + th_s[j] * thp_s[jp]);
  const double invP2 = 1.0 / ((double)P * P);
  std::vector<double> phip(J * FSZ), Kt(J * FSZ), psi(J * FSZ), psip(J * FSZ), psiw(J * FSZ),
      psips(J * FSZ);
  std::vector<double> phi_j(J);
  for (int kx = 0; kx < P; ++kx) {
    const double bx = centered_h(kx, P);
    for (int ky = 0; ky < P; ++ky) {
      const double by = centered_h(ky, P);
      const size_t o = colspec_index(kx, ky, E, TPR, NT);
      for (int j = 0; j < J; ++j) phi_j[j] = phi_R(bx * th_c[j] + by * th_s[j], L, R);
      for (int j = 0; j < J; ++j) {
        phip[j * FSZ + o] = phi_R(bx * thp_c[j] + by * thp_s[j], L, R);
        double k = 0.0;
        for (int i = 0; i < J; ++i) k += wG[(size_t)i * J + j] * phi_j[i];
        Kt[j * FSZ + o] = k * invP2;
        const double ps = psi_R(bx * th_c[j] + by * th_s[j], L, R);
        const double pp = psi_R(-bx * th_s[j] + by * th_c[j], L, R);  // theta_j rotated by pi/2
        psi[j * FSZ + o] = ps;
        psip[j * FSZ + o] = pp;
        psiw[j * FSZ + o] = (M_PI / J) * ps * invP2;
        psips[j * FSZ + o] = pp * invP2;
      }
    }
  }
  // col spec position of -k (mod P) for each position of k
  std::vector<unsigned> negk(FSZ);
  for (int kx = 0; kx < P; ++kx)
    for (int ky = 0; ky < P; ++ky)
      negk[colspec_index(kx, ky, E, TPR, NT)] = (unsigned)colspec_index((P - kx) % P, (P - ky) % P, E, TPR, NT);
  ts.built = put<T>(ts.tw, tw) && put<T>(ts.phip, phip) && put<T>(ts.Kt, Kt) && put<T>(ts.psi, psi) &&
             put<T>(ts.psip, psip) && put<T>(ts.psiw, psiw) && put<T>(ts.psips, psips) &&
             hip_ok(hipMemcpy(ts.negk, negk.data(), FSZ * sizeof(unsigned), hipMemcpyHostToDevice), "hipMemcpy");
  return ts.built;
}

// Index of tile shape E's table set, filled on first use (-1 on failure).
template <typename T>
int table_set(qb_plan_s* pl, int E) {
  int idx = -1;
  for (size_t i = 0; i < pl->tabs.size(); ++i)
    if (pl->tabs[i].E == E) idx = (int)i;
  if (idx < 0) return -1;
  if (!pl->tabs[idx].built && !fill_layout_tables<T>(pl, pl->tabs[idx])) return -1;
  return idx;
}

// Make tile shape E the reverse-mode pipeline's (0: follow the forward tile).
template <typename T>
bool select_vjp_tile(qb_plan_s* pl, int E) {
  const int idx = table_set<T>(pl, E > 0 ? E : pl->E);
  if (idx < 0) return false;
  pl->vjp_E = E;
  pl->vjp_tab = idx;
  return true;
}

// Make tile shape E current for the forward pipeline.
template <typename T>
bool select_tile(qb_plan_s* pl, int E) {
  const int idx = table_set<T>(pl, E);
  if (idx < 0) return false;
  pl->cur_tab = idx;
  if (pl->vjp_E == 0) pl->vjp_tab = idx;
  pl->E = E;
  pl->TPR = pl->P / E;
  pl->NT = pl->P * pl->TPR;
  // node pairing by default on every tile: its partner sums sit in registers,
  // or in buffer planes where the register plan has no room for them
  pl->i3_pair = true;
  return true;
}

// Gauss-Legendre weights and the separable modulation phases of
// eq. approxH-JM (natural frequency order, independent of the tile).
template <typename T>
bool reserve_phases(qb_plan_s* pl) {
  const size_t P = pl->P, J = pl->prob.J, M = pl->prob.M, b = sizeof(T);
  return pl->alloc(&pl->phx, J * M * P * 2 * b) && pl->alloc(&pl->phy, J * M * P * 2 * b) &&
         pl->alloc(&pl->wm, M * b);
}

template <typename T>
bool fill_phases(qb_plan_s* pl) {
  const qb_problem& p = pl->prob;
  const int P = pl->P, J = p.J, M = p.M;
  const double L = p.L, R = p.R;
  std::vector<double> th_c(J), th_s(J);
  for (int j = 0; j < J; ++j) {
    th_c[j] = std::cos(j * M_PI / J);
    th_s[j] = std::sin(j * M_PI / J);
  }
  std::vector<double> gx, gw;
  gauss_legendre(M, gx, gw);
  // the I_3 kernel pairs node m with M-1-m: make the symmetry exact
  for (int m = 0; m < M / 2; ++m) {
    const double x = 0.5 * (gx[M - 1 - m] - gx[m]), w = 0.5 * (gw[m] + gw[M - 1 - m]);
    gx[m] = -x;
    gx[M - 1 - m] = x;
    gw[m] = gw[M - 1 - m] = w;
  }
  if (M % 2 == 1) gx[M / 2] = 0.0;
  std::vector<double> phx((size_t)J * M * P * 2), phy((size_t)J * M * P * 2), wm(M);
  for (int m = 0; m < M; ++m) wm[m] = (M_PI / J) * R * gw[m];
  for (int j = 0; j < J; ++j)
    for (int m = 0; m < M; ++m) {
      const double rho = R * gx[m];
      for (int k = 0; k < P; ++k) {
        const double b = centered_h(k, P);
        const double ax = M_PI * rho * th_c[j] * b / L, ay = M_PI * rho * th_s[j] * b / L;
        const size_t o = (((size_t)j * M + m) * P + k) * 2;
        phx[o] = std::cos(ax);
        phx[o + 1] = std::sin(ax);
        phy[o] = std::cos(ay);
        phy[o + 1] = std::sin(ay);
      }
    }
  return put<T>(pl->phx, phx) && put<T>(pl->phy, phy) && put<T>(pl->wm, wm);
}

// Reserve the phases and one table set per compiled tile shape of the
// plan's padded grid.
template <typename T>
bool reserve_tables(qb_plan_s* pl) {
  if (!reserve_phases<T>(pl)) return false;
  for (int E : tile_candidates(pl->P)) {
    qb_plan_s::TabSet ts;
    if (!reserve_layout_tables<T>(pl, E, ts)) return false;
    pl->tabs.push_back(ts);
  }
  return true;
}

template <typename T>
bool fill_tables(qb_plan_s* pl) {
  return fill_phases<T>(pl) && select_tile<T>(pl, pl->E);
}

// Pauli components of W_FD (eq. W_FermiDirac) on the velocity grid: [4][N][N]
void fd_pauli(const qb_fd& s, int N, double L, double* out) {
  const double h = 2.0 * L / N;
  for (int i = 0; i < N; ++i)
    for (int j = 0; j < N; ++j) {
      const double vx = h * (i - N / 2), vy = h * (j - N / 2);
      const double om = 0.5 * (vx * vx + vy * vy);
      const double fu = 1.0 / (std::exp((om - s.mu_up) * s.inv_kT) + 1.0);
      const double fd = 1.0 / (std::exp((om - s.mu_down) * s.inv_kT) + 1.0);
      // W = U diag(fu, fd) U^H, U row-major
      double Wr[4], Wi[4];
      for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b) {
          double re = 0, im = 0;
          for (int c = 0; c < 2; ++c) {
            const double f = c == 0 ? fu : fd;
            const double ur = s.U_re[a * 2 + c], ui = s.U_im[a * 2 + c];
            const double vr = s.U_re[b * 2 + c], vi = -s.U_im[b * 2 + c];  // conj(U[b][c])
            re += f * (ur * vr - ui * vi);
            im += f * (ur * vi + ui * vr);
          }
          Wr[a * 2 + b] = re;
          Wi[a * 2 + b] = im;
        }
      const size_t o = (size_t)i * N + j, cs = (size_t)N * N;
      out[o] = 0.5 * (Wr[0] + Wr[3]);
      out[cs + o] = 0.5 * (Wr[2] + Wr[1]);
      out[2 * cs + o] = 0.5 * (Wi[2] - Wi[1]);
      out[3 * cs + o] = 0.5 * (Wr[0] - Wr[3]);
    }
}

// Wall tables of problem p (Dirichlet Phi or Maxwell W_FD on the velocity
// grid, the Maxwell normalization Z) carved from `owner`'s workspace: the
// device memory is reserved in every mode, and filled when not measuring.
template <typename T>
bool build_bc_for(qb_plan_s* owner, const qb_problem& p, qb::BcDev& bl, qb::BcDev& br, void** bcw, double** flux) {
  const int N = p.N;
  const size_t per = (size_t)N * N;
  if (!owner->alloc(bcw, 2 * 4 * per * sizeof(T)) || !owner->alloc((void**)flux, 2 * sizeof(double))) return false;
  std::vector<double> bw(2 * 4 * per, 0.0);
  const qb_bc* bcs[2] = {&p.left, &p.right};
  qb::BcDev* dv[2] = {&bl, &br};
  const double h = 2.0 * p.L / N;
  for (int wall = 0; wall < 2; ++wall) {
    const qb_bc& b = *bcs[wall];
    dv[wall]->kind = b.kind;
    dv[wall]->alpha = b.alpha;
    dv[wall]->Z = 1.0;
    if (b.kind == QB_PERIODIC || owner->measuring()) continue;
    double* o = bw.data() + wall * 4 * per;
    fd_pauli(b.state, N, p.L, o);
    if (b.kind == QB_MAXWELL) {
      // Z = h^2 sum over incoming (mirrored) rows of tr W_FD |v_x|
      double Z = 0.0;
      for (int i = 0; i < N; ++i) {
        const double vx = h * (i - N / 2);
        const bool in = wall == 0 ? vx > 0 : (vx < 0 && i != 0);
        if (!in) continue;
        for (int j = 0; j < N; ++j) Z += 2.0 * o[(size_t)i * N + j] * std::fabs(vx);
      }
      dv[wall]->Z = h * h * Z;
    }
  }
  if (owner->measuring()) return true;
  return put<T>(*bcw, bw) && hip_ok(hipMemset(*flux, 0, 2 * sizeof(double)), "hipMemset");
}

template <typename T>
bool build_bc(qb_plan_s* pl) {
  return build_bc_for<T>(pl, pl->prob, pl->bl, pl->br, &pl->bcw, &pl->flux);
}

// Per-cell buffers of the collision pipeline for `cells` cells per launch.
struct CollBufs {
  void *spec = nullptr, *wP = nullptr, *terms = nullptr, *acc = nullptr, *i3s = nullptr, *i3o = nullptr,
       *i3sum = nullptr, *i3p = nullptr, *i3ps = nullptr;
};

template <typename T>
bool carve_collision(Arena& a, const qb_plan_s* pl, size_t C, CollBufs& b) {
  const size_t FSZ = (size_t)pl->P * pl->P, J = pl->prob.J, t = sizeof(T);
  return a.take(&b.i3s, C * J * qb::kI3sPlanes<T> * FSZ * t) && a.take(&b.spec, C * 8 * FSZ * t) &&
         a.take(&b.wP, C * 5 * FSZ * t) && a.take(&b.terms, C * qb::kTermPlanes * FSZ * t) && a.take(&b.acc, C * 14 * FSZ * t) &&
         a.take(&b.i3o, C * J * 4 * FSZ * t) && a.take(&b.i3sum, C * 4 * FSZ * t) &&
         a.take(&b.i3p, C * J * 4 * FSZ * t) && a.take(&b.i3ps, C * 4 * FSZ * t);
}

CollBufs get_bufs(const qb_plan_s* pl) {
  CollBufs b;
  b.spec = pl->spec, b.wP = pl->wP, b.terms = pl->terms, b.acc = pl->acc, b.i3s = pl->i3s, b.i3o = pl->i3o;
  b.i3sum = pl->i3sum, b.i3p = pl->i3p, b.i3ps = pl->i3ps;
  return b;
}

void set_bufs(qb_plan_s* pl, const CollBufs& b) {
  pl->spec = b.spec, pl->wP = b.wP, pl->terms = b.terms, pl->acc = b.acc, pl->i3s = b.i3s, pl->i3o = b.i3o;
  pl->i3sum = b.i3sum, pl->i3p = b.i3p, pl->i3ps = b.i3ps;
}

template <typename T>
bool build_buffers(qb_plan_s* pl) {
  const qb_problem& p = pl->prob;
  const size_t st = (size_t)4 * p.Nx * p.N * p.N * sizeof(T);
  CollBufs b;
  if (!carve_collision<T>(pl->ws, pl, pl->wcells, b)) {
    set_error("plan workspace exhausted");
    return false;
  }
  set_bufs(pl, b);
  return pl->alloc(&pl->st0, st) && pl->alloc(&pl->st1, st) && pl->alloc(&pl->st2, st) && pl->alloc(&pl->cbuf, st);
}

template <typename T>
bool build_adjoint(qb_plan_s* pl) {
  const qb_problem& p = pl->prob;
  const size_t FSZ = (size_t)pl->P * pl->P, C = pl->wcells, J = p.J, b = sizeof(T);
  const size_t st = (size_t)4 * p.Nx * p.N * p.N * b;
  void** states[] = {&pl->wn, &pl->wa, &pl->w1, &pl->wb, &pl->lb, &pl->ls, &pl->la, &pl->cg, &pl->g0};
  for (void** q : states)
    if (!pl->alloc_adj(q, st)) return false;
  return pl->alloc_adj(&pl->lamP, C * 4 * FSZ * b) && pl->alloc_adj(&pl->acot, C * 16 * FSZ * b) &&
         pl->alloc_adj(&pl->gspec, C * 22 * FSZ * b) && pl->alloc_adj(&pl->gf0, C * 7 * FSZ * b) &&
         pl->alloc_adj(&pl->i3g, C * J * 8 * FSZ * b) && pl->alloc_adj(&pl->i3sb, C * J * 4 * FSZ * b) &&
         pl->alloc_adj(&pl->gsum, C * 8 * FSZ * b) && pl->alloc_adj(&pl->i3t, C * J * 4 * FSZ * b) &&
         pl->alloc_adj(&pl->lamh, C * 4 * FSZ * b) && pl->alloc_adj(&pl->fwa, C * 14 * FSZ * b) &&
         pl->alloc_adj(&pl->ext, (size_t)4 * (p.Nx + 4) * p.N * p.N * b) &&
         pl->alloc_adj((void**)&pl->lflux, 2 * sizeof(double));
}


template <typename T>
bool collision_chunk(qb_plan_s* pl, const T* w, T* c, int ncells, int cell0, hipStream_t s) {
  switch (pl->P) {
    case 32:
      return pl->E == 8 ? collision_pipeline<T, 32, 8>(pl, w, c, ncells, cell0, s)
                        : collision_pipeline<T, 32, 16>(pl, w, c, ncells, cell0, s);
    case 64:
      return pl->E == 16  ? collision_pipeline<T, 64, 16>(pl, w, c, ncells, cell0, s)
             : pl->E == 8 ? collision_pipeline<T, 64, 8>(pl, w, c, ncells, cell0, s)
                          : collision_pipeline<T, 64, 32>(pl, w, c, ncells, cell0, s);
    case 128:
      return pl->E == 16 ? collision_pipeline<T, 128, 16>(pl, w, c, ncells, cell0, s)
                         : collision_pipeline<T, 128, 32>(pl, w, c, ncells, cell0, s);
  }
  return false;
}

// C[w] for cells [0, ncells), in chunks of at most wcells cells
template <typename T>
bool collision_any(qb_plan_s* pl, const T* w, T* c, int ncells, hipStream_t s) {
  for (int c0 = 0; c0 < ncells; c0 += pl->wcells)
    if (!collision_chunk<T>(pl, w, c, std::min(pl->wcells, ncells - c0), c0, s)) return false;
  return true;
}

// Boundary data of one problem's cells inside a state array: the first
// cell, the cell count, the walls and their device tables.
struct Segment {
  int offset, Nx;
  qb::BcDev bl, br;
  const void* bcw;
  double* flux;
  bool left_maxwell, right_maxwell;
};

Segment whole(qb_plan_s* pl) {
  const qb_problem& p = pl->prob;
  return Segment{0, p.Nx, pl->bl, pl->br, pl->bcw, pl->flux, p.left.kind == QB_MAXWELL, p.right.kind == QB_MAXWELL};
}

// tmp = T(dt) cur on one segment; arrays hold `ntot` cells per component
template <typename T>
void transport_seg(qb_plan_s* pl, const T* cur, T* tmp, double dt, const Segment& g, int ntot, hipStream_t s) {
  const int N = pl->prob.N;
  const size_t per = (size_t)N * N, n = (size_t)g.Nx * per, off = (size_t)g.offset * per;
  const int lm = g.left_maxwell, rm = g.right_maxwell;
  if (lm || rm)
    hipLaunchKernelGGL((qb::k_maxwell_flux<T>), dim3(2), dim3(256), 0, s, cur + off, g.flux, g.Nx, N, pl->prob.L, lm,
                       rm);
  hipLaunchKernelGGL((qb::k_transport<T>), dim3(blocks(n, 256)), dim3(256), 0, s, cur + off, tmp + off,
                     (const T*)g.bcw, g.flux, g.bl, g.br, (T)dt, g.Nx, N, (T)pl->prob.L, ntot, pl->limiter);
}

// Net inflow through the two walls during one transport step of length dt,
// from the flux form of eq. slopeLimiterStep, W_j <- W_j - (dt/dx)
// (F_{j+1/2} - F_{j-1/2}) with
//   F_{j+1/2} = (v (W_j + W_{j+1}) - |v| (W_{j+1} - W_j)) / 2
//             + l (v (S_j + S_{j+1}) - |v| (S_{j+1} - S_j)) / 2,
// l = (sgn nu - nu) / 2, in the units of the cell-summed moments:
// (dt/dx) h^2 sum_v phi(v) (F_{1/2} - F_{Nx+1/2}) for phi = (rho_0..3,
// v_x tr, v_y tr, |v|^2/2 tr); written to out[0..6], or added to it.
// One workgroup of 256 threads.
template <typename T>
__global__ __launch_bounds__(256) void k_wall_inflow(const T* __restrict__ w, const T* __restrict__ bcw,
                                                     const double* __restrict__ flux, qb::BcDev bl, qb::BcDev br, T dt,
                                                     int Nx, int N, T L, int Ntot, int limiter,
                                                     double* __restrict__ out, int accumulate) {
  const int per = N * N;
  const size_t cs = (size_t)Ntot * per;
  const T h = (T)2 * L / (T)N;
  const T dx = (T)1 / (T)Nx;
  double acc[7] = {0, 0, 0, 0, 0, 0, 0};
  for (int e = threadIdx.x; e < per; e += blockDim.x) {
    const int i = e / N;
    const T vx = h * (T)(i - N / 2), vy = h * (T)(e % N - N / 2);
    const T nu = dt * vx / dx;
    const T sg = vx > (T)0 ? (T)1 : (vx < (T)0 ? (T)-1 : (T)0);
    const T lim = (T)0.5 * (sg - nu);
    const T av = fabs(vx);
    for (int mu = 0; mu < 4; ++mu) {
      T F[2];
      for (int side = 0; side < 2; ++side) {
        // cells c0 .. c0 + 3 around the face between c0 + 1 and c0 + 2
        const int c0 = side == 0 ? -2 : Nx - 2;
        T g[4];
        for (int k = 0; k < 4; ++k) g[k] = qb::ext_value(w, bcw, flux, bl, br, mu, c0 + k, e, i, vx, Nx, N, cs);
        const T Sa = qb::slope(limiter, g[2] - g[1], g[1] - g[0]);
        const T Sb = qb::slope(limiter, g[3] - g[2], g[2] - g[1]);
        F[side] = (T)0.5 * (vx * (g[1] + g[2]) - av * (g[2] - g[1])) +
                  (T)0.5 * lim * (vx * (Sa + Sb) - av * (Sb - Sa));
      }
      const double net = (double)F[0] - (double)F[1];
      acc[mu] += net;
      if (mu == 0) {
        acc[4] += (double)vx * 2.0 * net;
        acc[5] += (double)vy * 2.0 * net;
        acc[6] += 0.5 * ((double)vx * vx + (double)vy * vy) * 2.0 * net;
      }
    }
  }
  __shared__ double red[7][256];
  for (int k = 0; k < 7; ++k) red[k][threadIdx.x] = acc[k];
  __syncthreads();
  for (int o = blockDim.x / 2; o > 0; o >>= 1) {
    if (threadIdx.x < o)
      for (int k = 0; k < 7; ++k) red[k][threadIdx.x] += red[k][threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x < 7) {
    const double sc = (double)dt * Nx * (double)h * (double)h;
    const double v = sc * red[threadIdx.x][0];
    out[threadIdx.x] = accumulate ? out[threadIdx.x] + v : v;
  }
}

// out[0..6] (= or +=) the moments of the net inflow through the walls
// during the transport step of length dt that is about to run on cur
template <typename T>
bool wall_inflow(qb_plan_s* pl, const T* cur, double dt, double* out, bool accumulate, hipStream_t s) {
  const Segment g = whole(pl);
  const int N = pl->prob.N;
  if (g.left_maxwell || g.right_maxwell)
    hipLaunchKernelGGL((qb::k_maxwell_flux<T>), dim3(2), dim3(256), 0, s, cur, g.flux, g.Nx, N, pl->prob.L,
                       (int)g.left_maxwell, (int)g.right_maxwell);
  hipLaunchKernelGGL((k_wall_inflow<T>), dim3(1), dim3(256), 0, s, cur, (const T*)g.bcw, g.flux, g.bl, g.br,
                     (T)dt, g.Nx, N, (T)pl->prob.L, g.Nx, pl->limiter, out, accumulate ? 1 : 0);
  return hip_ok(hipGetLastError(), "wall inflow launch");
}

template <typename T>
bool transport(qb_plan_s* pl, T*& cur, T*& tmp, double dt, hipStream_t s) {
  const int id = pl->begin(QB_K_TRANSPORT, s);
  transport_seg<T>(pl, cur, tmp, dt, whole(pl), pl->prob.Nx, s);
  pl->end(id, s);
  std::swap(cur, tmp);
  return hip_ok(hipGetLastError(), "transport launch");
}

// dst = T(dt) src (src unchanged)
template <typename T>
bool transport_to(qb_plan_s* pl, const T* src, T* dst, double dt, hipStream_t s) {
  T* a = (T*)src;
  T* b = dst;
  return transport<T>(pl, a, b, dt, s);
}

// ------------------------------------------------------------------ adjoint pipelines
template <typename T>
bool collision_vjp_chunk(qb_plan_s* pl, const T* w, const T* lam, T* out, int n, int c0, hipStream_t s) {
  const int E = pl->tabs[pl->vjp_tab].E;  // the reverse-mode tile
  switch (pl->P) {
    case 32:
      return E == 8 ? collision_vjp_pipeline<T, 32, 8>(pl, w, lam, out, n, c0, s)
                    : collision_vjp_pipeline<T, 32, 16>(pl, w, lam, out, n, c0, s);
    case 64:
      return E == 16  ? collision_vjp_pipeline<T, 64, 16>(pl, w, lam, out, n, c0, s)
             : E == 8 ? collision_vjp_pipeline<T, 64, 8>(pl, w, lam, out, n, c0, s)
                      : collision_vjp_pipeline<T, 64, 32>(pl, w, lam, out, n, c0, s);
    case 128:
      return E == 16 ? collision_vjp_pipeline<T, 128, 16>(pl, w, lam, out, n, c0, s)
                     : collision_vjp_pipeline<T, 128, 32>(pl, w, lam, out, n, c0, s);
  }
  return false;
}

template <typename T>
bool collision_vjp_any(qb_plan_s* pl, const T* w, const T* lam, T* out, int ncells, hipStream_t s) {
  for (int c0 = 0; c0 < ncells; c0 += pl->wcells)
    if (!collision_vjp_chunk<T>(pl, w, lam, out, std::min(pl->wcells, ncells - c0), c0, s)) return false;
  return true;
}

// out = T'(x)^T lam for one transport step of length dt taken at state x
template <typename T>
bool transport_vjp(qb_plan_s* pl, const T* x, const T* lam, T* out, double dt, hipStream_t s) {
  const qb_problem& p = pl->prob;
  const int lm = p.left.kind == QB_MAXWELL, rm = p.right.kind == QB_MAXWELL;
  const size_t n = (size_t)p.Nx * p.N * p.N, ne = (size_t)(p.Nx + 4) * p.N * p.N;
  const int id = pl->begin(QB_K_ADJOINT, s);
  if (lm || rm) hipLaunchKernelGGL((qb::k_maxwell_flux<T>), dim3(2), dim3(256), 0, s, x, pl->flux, p.Nx, p.N, p.L, lm, rm);
  hipLaunchKernelGGL((qb::k_transport_vjp_ext<T>), dim3(blocks(ne, 256)), dim3(256), 0, s, x, lam, (T*)pl->ext,
                     (const T*)pl->bcw, pl->flux, pl->bl, pl->br, (T)dt, p.Nx, p.N, (T)p.L);
  if (lm || rm)
    hipLaunchKernelGGL((qb::k_maxwell_lflux<T>), dim3(2), dim3(256), 0, s, (const T*)pl->ext, (const T*)pl->bcw,
                       pl->lflux, pl->bl, pl->br, p.Nx, p.N);
  hipLaunchKernelGGL((qb::k_transport_vjp_fold<T>), dim3(blocks(n, 256)), dim3(256), 0, s, (const T*)pl->ext, out,
                     pl->lflux, pl->bl, pl->br, p.Nx, p.N, (T)p.L);
  pl->end(id, s);
  return hip_ok(hipGetLastError(), "transport adjoint launch");
}

template <typename T>
bool moments(qb_plan_s* pl, const T* w, double* mom, hipStream_t s) {
  const qb_problem& p = pl->prob;
  const int id = pl->begin(QB_K_MOMENTS, s);
  hipLaunchKernelGGL((qb::k_moments<T>), dim3(p.Nx), dim3(256), 0, s, w, mom, p.Nx, p.N, p.L);
  pl->end(id, s);
  return hip_ok(hipGetLastError(), "moments launch");
}

template <typename T, typename TA>
bool to_state(qb_plan_s* pl, const void* W, T* w, int ncells, hipStream_t s) {
  const qb_problem& p = pl->prob;
  const size_t n = (size_t)ncells * p.N * p.N;
  hipLaunchKernelGGL((qb::k_api_to_state<T, TA>), dim3(blocks(n, 256)), dim3(256), 0, s, (const TA*)W, w, ncells,
                     p.N, p.Nx);
  return hip_ok(hipGetLastError(), "layout launch");
}
template <typename T, typename TA>
bool from_state(qb_plan_s* pl, const T* w, void* W, int ncells, hipStream_t s) {
  const qb_problem& p = pl->prob;
  const size_t n = (size_t)ncells * p.N * p.N;
  hipLaunchKernelGGL((qb::k_state_to_api<T, TA>), dim3(blocks(n, 256)), dim3(256), 0, s, w, (TA*)W, ncells, p.N,
                     p.Nx);
  return hip_ok(hipGetLastError(), "layout launch");
}

template <typename T>
bool to_cot(qb_plan_s* pl, const void* G, T* g, int ncells, hipStream_t s) {
  const qb_problem& p = pl->prob;
  const size_t n = (size_t)ncells * p.N * p.N;
  hipLaunchKernelGGL((qb::k_api_to_cot<T, T>), dim3(blocks(n, 256)), dim3(256), 0, s, (const T*)G, g, ncells, p.N,
                     p.Nx);
  return hip_ok(hipGetLastError(), "layout launch");
}
template <typename T>
bool from_cot(qb_plan_s* pl, const T* g, void* G, int ncells, hipStream_t s) {
  const qb_problem& p = pl->prob;
  const size_t n = (size_t)ncells * p.N * p.N;
  hipLaunchKernelGGL((qb::k_cot_to_api<T, T>), dim3(blocks(n, 256)), dim3(256), 0, s, g, (T*)G, ncells, p.N, p.Nx);
  return hip_ok(hipGetLastError(), "layout launch");
}

template <typename T>
qb_status do_collision(qb_plan_s* pl, const void* W, void* C, int ncells, hipStream_t s) {
  T* w = (T*)pl->st0;
  T* c = (T*)pl->cbuf;
  if (!to_state<T, T>(pl, W, w, ncells, s)) return QB_EHIP;
  if (!collision_any<T>(pl, w, c, ncells, s)) return QB_EHIP;
  if (!from_state<T, T>(pl, c, C, ncells, s)) return QB_EHIP;
  return QB_OK;
}

template <typename T>
qb_status do_step(qb_plan_s* pl, void* W, const double* B, double dt, int nsteps, double* mom, T* trace,
                  hipStream_t s, double* inflow = nullptr) {
  const qb_problem& p = pl->prob;
  T* cur = (T*)pl->st0;
  T* tmp = (T*)pl->st2;
  T* w1 = (T*)pl->st1;
  T* c = (T*)pl->cbuf;
  const size_t n = (size_t)p.Nx * p.N * p.N;
  const size_t mstride = (size_t)p.Nx * 7;
  if (!to_state<T, T>(pl, W, cur, p.Nx, s)) return QB_EHIP;
  if (mom && !moments<T>(pl, cur, mom, s)) return QB_EHIP;
  const size_t sb = 4 * n * sizeof(T);
  for (int it = 0; it < nsteps; ++it) {
    // trace record of this step: [step input, Heun stage 1, Heun output]
    T* rec = trace ? trace + (size_t)it * 3 * 4 * n : nullptr;
    if (rec && !hip_ok(hipMemcpyAsync(rec, cur, sb, hipMemcpyDeviceToDevice, s), "trace copy")) return QB_EHIP;
    if (inflow && !wall_inflow<T>(pl, cur, 0.5 * dt, inflow + (size_t)it * 7, false, s)) return QB_EHIP;
    if (!transport<T>(pl, cur, tmp, 0.5 * dt, s)) return QB_EHIP;
    // field term: inside the Heun step, or its exact flow for dt/2 on
    // either side of a collision-only Heun step
    const bool rot = pl->field_mode == QB_FIELD_ROTATION && B;
    const double* Bh = rot ? nullptr : B;
    if (rot) {
      const int rid = pl->begin(QB_K_HEUN, s);
      hipLaunchKernelGGL((qb::k_rotate<T>), dim3(blocks(n, 256)), dim3(256), 0, s, cur, B, 0.5 * dt, p.Nx, p.N);
      pl->end(rid, s);
    }
    if (!collision_any<T>(pl, cur, c, p.Nx, s)) return QB_EHIP;
    int id = pl->begin(QB_K_HEUN, s);
    hipLaunchKernelGGL((qb::k_heun<T>), dim3(blocks(n, 256)), dim3(256), 0, s, cur, w1, c, Bh, (T)dt, p.Nx, p.N, 1);
    pl->end(id, s);
    if (rec && !hip_ok(hipMemcpyAsync(rec + 4 * n, w1, sb, hipMemcpyDeviceToDevice, s), "trace copy"))
      return QB_EHIP;
    if (!collision_any<T>(pl, w1, c, p.Nx, s)) return QB_EHIP;
    id = pl->begin(QB_K_HEUN, s);
    hipLaunchKernelGGL((qb::k_heun<T>), dim3(blocks(n, 256)), dim3(256), 0, s, cur, w1, c, Bh, (T)dt, p.Nx, p.N, 2);
    pl->end(id, s);
    if (rot) {
      const int rid = pl->begin(QB_K_HEUN, s);
      hipLaunchKernelGGL((qb::k_rotate<T>), dim3(blocks(n, 256)), dim3(256), 0, s, cur, B, 0.5 * dt, p.Nx, p.N);
      pl->end(rid, s);
    }
    if (!hip_ok(hipGetLastError(), "heun launch")) return QB_EHIP;
    if (rec && !hip_ok(hipMemcpyAsync(rec + 8 * n, cur, sb, hipMemcpyDeviceToDevice, s), "trace copy"))
      return QB_EHIP;
    if (inflow && !wall_inflow<T>(pl, cur, 0.5 * dt, inflow + (size_t)it * 7, true, s)) return QB_EHIP;
    if (!transport<T>(pl, cur, tmp, 0.5 * dt, s)) return QB_EHIP;
    if (mom && !moments<T>(pl, cur, mom + (it + 1) * mstride, s)) return QB_EHIP;
  }
  if (!from_state<T, T>(pl, cur, W, p.Nx, s)) return QB_EHIP;
  // keep st0 as the home of the state for the next call
  if (cur != (T*)pl->st0) std::swap(pl->st0, pl->st2);
  return QB_OK;
}

template <typename T>
qb_status do_transport(qb_plan_s* pl, void* W, double dt, hipStream_t s) {
  const qb_problem& p = pl->prob;
  T* cur = (T*)pl->st0;
  T* tmp = (T*)pl->st2;
  if (!to_state<T, T>(pl, W, cur, p.Nx, s)) return QB_EHIP;
  if (!transport<T>(pl, cur, tmp, dt, s)) return QB_EHIP;
  if (!from_state<T, T>(pl, cur, W, p.Nx, s)) return QB_EHIP;
  if (cur != (T*)pl->st0) std::swap(pl->st0, pl->st2);
  return QB_OK;
}

template <typename T>
qb_status do_moments(qb_plan_s* pl, const void* W, double* mom, hipStream_t s) {
  T* cur = (T*)pl->st0;
  if (!to_state<T, T>(pl, W, cur, pl->prob.Nx, s)) return QB_EHIP;
  if (!moments<T>(pl, cur, mom, s)) return QB_EHIP;
  return QB_OK;
}

template <typename T>
qb_status do_diagnostics(qb_plan_s* pl, const void* W, const void* C, const qb::FdGlobal& g, double* out,
                         hipStream_t s) {
  const qb_problem& p = pl->prob;
  const int id = pl->begin(QB_K_DIAGNOSTICS, s);
  hipLaunchKernelGGL((qb::k_diagnostics<T>), dim3(p.Nx), dim3(256), 0, s, (const T*)W, (const T*)C, g, out, p.N, p.L);
  pl->end(id, s);
  return hip_ok(hipGetLastError(), "diagnostics launch") ? QB_OK : QB_EHIP;
}

template <typename T>
qb_status do_collision_vjp(qb_plan_s* pl, const void* W, const void* lam, void* G, int ncells, hipStream_t s) {
  T* w = (T*)pl->wn;
  T* g = (T*)pl->g0;
  T* out = (T*)pl->cg;
  if (!to_state<T, T>(pl, W, w, ncells, s) || !to_cot<T>(pl, lam, g, ncells, s)) return QB_EHIP;
  if (!collision_vjp_any<T>(pl, w, g, out, ncells, s)) return QB_EHIP;
  return from_cot<T>(pl, out, G, ncells, s) ? QB_OK : QB_EHIP;
}

template <typename T>
qb_status do_transport_vjp(qb_plan_s* pl, const void* W, double dt, const void* lam, void* G, hipStream_t s) {
  const int Nx = pl->prob.Nx;
  T* w = (T*)pl->wn;
  T* g = (T*)pl->g0;
  T* out = (T*)pl->lb;
  if (!to_state<T, T>(pl, W, w, Nx, s) || !to_cot<T>(pl, lam, g, Nx, s)) return QB_EHIP;
  if (!transport_vjp<T>(pl, w, g, out, dt, s)) return QB_EHIP;
  return from_cot<T>(pl, out, G, Nx, s) ? QB_OK : QB_EHIP;
}

// Reverse of one splitting step S = T(dt/2) . Heun(dt) . T(dt/2):
//   lam_b = T'(wb)^T lam_next
//   lam_1 = lam_b / 2 + dt/2 F'(w1)^T lam_b
//   lam_a = lam_b / 2 + lam_1 + dt F'(wa)^T lam_1
//   lam   = T'(wn)^T lam_a
// with wn the step input, wa = T(dt/2) wn, w1 the Heun stage and wb the Heun
// output (taken from the trace record, or recomputed here).
template <typename T>
qb_status do_adjoint_step(qb_plan_s* pl, const void* W, const void* record, const double* B, double dt,
                          const void* lam_next, void* lam, double* gB, hipStream_t s) {
  const qb_problem& p = pl->prob;
  const size_t n = (size_t)p.Nx * p.N * p.N;
  const size_t sb = 4 * n * sizeof(T);
  T *wn, *w1, *wb;
  T* wa = (T*)pl->wa;
  T* c = (T*)pl->cbuf;
  if (record) {
    wn = (T*)record;
    w1 = wn + 4 * n;
    wb = wn + 8 * n;
    if (!transport_to<T>(pl, wn, wa, 0.5 * dt, s)) return QB_EHIP;
  } else {
    wn = (T*)pl->wn;
    w1 = (T*)pl->w1;
    wb = (T*)pl->wb;
    if (!to_state<T, T>(pl, W, wn, p.Nx, s)) return QB_EHIP;
    if (!transport_to<T>(pl, wn, wa, 0.5 * dt, s)) return QB_EHIP;
    if (!collision_any<T>(pl, wa, c, p.Nx, s)) return QB_EHIP;
    hipLaunchKernelGGL((qb::k_heun<T>), dim3(blocks(n, 256)), dim3(256), 0, s, wa, w1, c, B, (T)dt, p.Nx, p.N, 1);
    if (!hip_ok(hipMemcpyAsync(wb, wa, sb, hipMemcpyDeviceToDevice, s), "copy")) return QB_EHIP;
    if (!collision_any<T>(pl, w1, c, p.Nx, s)) return QB_EHIP;
    hipLaunchKernelGGL((qb::k_heun<T>), dim3(blocks(n, 256)), dim3(256), 0, s, wb, w1, c, B, (T)dt, p.Nx, p.N, 2);
    if (!hip_ok(hipGetLastError(), "heun launch")) return QB_EHIP;
  }
  T* g0 = (T*)pl->g0;
  T* lb = (T*)pl->lb;
  T* l1 = (T*)pl->ls;
  T* la = (T*)pl->la;
  T* cg = (T*)pl->cg;
  if (!to_cot<T>(pl, lam_next, g0, p.Nx, s)) return QB_EHIP;
  if (!transport_vjp<T>(pl, wb, g0, lb, 0.5 * dt, s)) return QB_EHIP;
  if (!collision_vjp_any<T>(pl, w1, lb, cg, p.Nx, s)) return QB_EHIP;
  int id = pl->begin(QB_K_ADJOINT, s);
  hipLaunchKernelGGL((qb::k_heun_vjp<T>), dim3(p.Nx), dim3(256), 0, s, lb, (const T*)nullptr, cg, w1, B, l1, gB,
                     (T)dt, p.Nx, p.N, 2);
  pl->end(id, s);
  if (!collision_vjp_any<T>(pl, wa, l1, cg, p.Nx, s)) return QB_EHIP;
  id = pl->begin(QB_K_ADJOINT, s);
  hipLaunchKernelGGL((qb::k_heun_vjp<T>), dim3(p.Nx), dim3(256), 0, s, lb, l1, cg, wa, B, la, gB, (T)dt, p.Nx, p.N,
                     1);
  pl->end(id, s);
  if (!hip_ok(hipGetLastError(), "heun adjoint launch")) return QB_EHIP;
  if (!transport_vjp<T>(pl, wn, la, g0, 0.5 * dt, s)) return QB_EHIP;
  return from_cot<T>(pl, g0, lam, p.Nx, s) ? QB_OK : QB_EHIP;
}

// ------------------------------------------------------------------ tuning
// Time the collision pipeline on `ncells` cells for every tile shape of the
// plan's padded grid and keep the fastest; choices are cached per (precision,
// N, J, M, ncells) for the life of the process.
struct TuneKey {
  int precision, N, J, M, ncells;
  bool operator<(const TuneKey& o) const {
    return std::tie(precision, N, J, M, ncells) < std::tie(o.precision, o.N, o.J, o.M, o.ncells);
  }
};
std::map<TuneKey, int>& tune_cache() {
  static std::map<TuneKey, int> m;
  return m;
}

template <typename T>
qb_status do_tune(qb_plan_s* pl, int ncells, int* chosen, hipStream_t s) {
  const qb_problem& p = pl->prob;
  const std::vector<int> cands = tile_candidates(pl->P);
  const TuneKey key{p.precision, p.N, p.J, p.M, ncells};
  auto it = tune_cache().find(key);
  int best = cands[0];
  bool best_pair = true;
  if (it != tune_cache().end()) {
    best = it->second / 2;
    best_pair = it->second % 2 == 1;
  } else {
    T* w = (T*)pl->st0;
    T* c = (T*)pl->cbuf;
    if (!hip_ok(hipMemsetAsync(w, 0, (size_t)4 * p.Nx * p.N * p.N * sizeof(T), s), "hipMemsetAsync"))
      return QB_EHIP;
    const bool prof = pl->profiling;
    pl->profiling = false;
    hipEvent_t a = pl->event(), b = pl->event();
    float best_ms = 1e30f;
    for (int E : cands)
      for (int pair = 0; pair < 2; ++pair) {
        if (!select_tile<T>(pl, E)) return QB_EHIP;
        pl->i3_pair = pair == 1;
        if (!collision_any<T>(pl, w, c, ncells, s)) return QB_EHIP;  // warm-up
        (void)hipEventRecord(a, s);
        for (int r = 0; r < 2; ++r)
          if (!collision_any<T>(pl, w, c, ncells, s)) return QB_EHIP;
        (void)hipEventRecord(b, s);
        if (!hip_ok(hipEventSynchronize(b), "hipEventSynchronize")) return QB_EHIP;
        float ms = 0.f;
        (void)hipEventElapsedTime(&ms, a, b);
        if (ms < best_ms) {
          best_ms = ms;
          best = E;
          best_pair = pair == 1;
        }
      }
    pl->pool.push_back(a);
    pl->pool.push_back(b);
    pl->profiling = prof;
    tune_cache()[key] = 2 * best + (best_pair ? 1 : 0);
  }
  if (!select_tile<T>(pl, best)) return QB_EHIP;
  pl->i3_pair = best_pair;
  if (chosen) *chosen = best;
  {
    // one workgroup per task against a persistent grid of resident
    // workgroups striding over the tasks (same kernels, same results)
    const TuneKey pkey{p.precision + 32, p.N, p.J, p.M, ncells};
    auto pt = tune_cache().find(pkey);
    if (pt != tune_cache().end()) {
      pl->persistent = pt->second == 1;
    } else {
      T* w = (T*)pl->st0;
      T* c = (T*)pl->cbuf;
      if (!hip_ok(hipMemsetAsync(w, 0, (size_t)4 * p.Nx * p.N * p.N * sizeof(T), s), "hipMemsetAsync"))
        return QB_EHIP;
      const bool prof = pl->profiling;
      pl->profiling = false;
      hipEvent_t a = pl->event(), b = pl->event();
      float t[2] = {0.f, 0.f};
      for (int v = 0; v < 2; ++v) {
        pl->persistent = v == 1;
        if (!collision_any<T>(pl, w, c, ncells, s)) return QB_EHIP;  // warm-up
        (void)hipEventRecord(a, s);
        for (int r = 0; r < 2; ++r)
          if (!collision_any<T>(pl, w, c, ncells, s)) return QB_EHIP;
        (void)hipEventRecord(b, s);
        if (!hip_ok(hipEventSynchronize(b), "hipEventSynchronize")) return QB_EHIP;
        (void)hipEventElapsedTime(&t[v], a, b);
      }
      pl->pool.push_back(a);
      pl->pool.push_back(b);
      pl->profiling = prof;
      // the two shapes tie within the timing noise on launches that fill the
      // machine; the persistent grid has to win by more than 1 %
      pl->persistent = t[1] < 0.99f * t[0];
      tune_cache()[pkey] = pl->persistent ? 1 : 0;
    }
  }
  if (pl->adjoint) {
    // the reverse-mode pipeline: every tile shape (its own table set) and
    // both I_3 adjoint kernels; the choice is cached as 16 E + variant
    const TuneKey vkey{p.precision + 16, p.N, p.J, p.M, ncells};
    auto vt = tune_cache().find(vkey);
    int vE = best, vv = 0;
    if (vt != tune_cache().end()) {
      vE = vt->second / 16;
      vv = vt->second % 16;
    } else {
      T* w = (T*)pl->st0;
      T* g = (T*)pl->g0;
      T* out = (T*)pl->cg;
      const size_t n = (size_t)4 * p.Nx * p.N * p.N * sizeof(T);
      if (!hip_ok(hipMemsetAsync(w, 0, n, s), "hipMemsetAsync") || !hip_ok(hipMemsetAsync(g, 0, n, s), "hipMemsetAsync"))
        return QB_EHIP;
      const bool prof = pl->profiling;
      pl->profiling = false;
      hipEvent_t a = pl->event(), b = pl->event();
      float best_ms = 1e30f;
      for (int E : cands)
        for (int v = 0; v < 2; ++v) {
          if (!select_vjp_tile<T>(pl, E)) return QB_EHIP;
          pl->vjp_variant = v;
          if (!collision_vjp_any<T>(pl, w, g, out, ncells, s)) return QB_EHIP;
          (void)hipEventRecord(a, s);
          if (!collision_vjp_any<T>(pl, w, g, out, ncells, s)) return QB_EHIP;
          (void)hipEventRecord(b, s);
          if (!hip_ok(hipEventSynchronize(b), "hipEventSynchronize")) return QB_EHIP;
          float ms = 0.f;
          (void)hipEventElapsedTime(&ms, a, b);
          if (ms < best_ms) {
            best_ms = ms;
            vE = E;
            vv = v;
          }
        }
      pl->pool.push_back(a);
      pl->pool.push_back(b);
      pl->profiling = prof;
      tune_cache()[vkey] = 16 * vE + vv;
    }
    if (!select_vjp_tile<T>(pl, vE)) return QB_EHIP;
    pl->vjp_variant = vv;
  }
  return QB_OK;
}

qb_status validate_bc(const qb_bc& b) {
  if (b.kind != QB_PERIODIC && b.kind != QB_DIRICHLET && b.kind != QB_MAXWELL) return QB_EINVAL;
  if (b.kind == QB_MAXWELL && !(b.alpha >= 0.0 && b.alpha <= 1.0)) return QB_EINVAL;
  if (b.kind != QB_PERIODIC && !(b.state.inv_kT > 0.0)) return QB_EINVAL;
  return QB_OK;
}

qb_status validate(const qb_problem* p) {
  if (!p) return QB_EINVAL;
  if (p->Nx < 1 || p->J < 1 || p->M < 1 || !(p->L > 0.0) || !(p->R >= 0.0)) return QB_EINVAL;
  if (p->precision != QB_F64 && p->precision != QB_F32) return QB_EINVAL;
  if (p->N != 16 && p->N != 32 && p->N != 64) return QB_ENOTSUP;
  if ((p->J % 2) != 0 || p->J > 128 || p->M > 256) return QB_ENOTSUP;
  qb_status s = validate_bc(p->left);
  if (s != QB_OK) return s;
  s = validate_bc(p->right);
  if (s != QB_OK) return s;
  if ((p->left.kind == QB_PERIODIC) != (p->right.kind == QB_PERIODIC)) return QB_EINVAL;
  return QB_OK;
}

// Default number of cells one collision launch covers: the collision
// workspace (about (43 + 12 J) P^2 scalars per cell) is sized for this many.
constexpr int kChunkCells = 512;

int chunk_cells(const qb_problem& p, int max_cells) {
  return std::min(p.Nx, max_cells > 0 ? max_cells : kChunkCells);
}

void init_plan(qb_plan_s* pl, const qb_problem& problem, int max_cells) {
  pl->prob = problem;
  pl->P = 2 * problem.N;
  pl->E = cfg_E(problem.precision, pl->P);
  pl->TPR = pl->P / pl->E;
  pl->NT = pl->P * pl->TPR;
  pl->wcells = chunk_cells(problem, max_cells);
}

// Carve (and, unless measuring, fill) everything a plan holds: phases and
// the table set of every tile shape, wall tables, collision and state
// buffers.  The same code sizes the workspace (measuring) and builds it.
template <typename T>
bool layout_plan(qb_plan_s* pl) {
  if (!reserve_tables<T>(pl) || !build_bc<T>(pl) || !build_buffers<T>(pl)) return false;
  return pl->measuring() || fill_tables<T>(pl);
}

bool layout_any(qb_plan_s* pl) {
  return pl->prob.precision == QB_F64 ? layout_plan<double>(pl) : layout_plan<float>(pl);
}

size_t plan_workspace_bytes(const qb_problem& problem, int max_cells) {
  qb_plan_s pl;
  init_plan(&pl, problem, max_cells);
  pl.ws.reset(nullptr, 0, true);
  return layout_any(&pl) ? pl.ws.used : 0;
}

qb_plan_s* create_plan(const qb_problem& problem, int max_cells, void* ws, size_t ws_bytes) {
  qb_plan_s* pl = new qb_plan_s();
  init_plan(pl, problem, max_cells);
  pl->ws.reset(ws, ws_bytes, false);
  if (!layout_any(pl)) {
    delete pl;
    return nullptr;
  }
  return pl;
}

size_t adjoint_workspace_bytes(qb_plan_s* pl) {
  const Arena keep = pl->adj;
  pl->adj.reset(nullptr, 0, true);
  const bool ok = pl->prob.precision == QB_F64 ? build_adjoint<double>(pl) : build_adjoint<float>(pl);
  const size_t n = pl->adj.used;
  pl->adj = keep;
  return ok ? n : 0;
}

}  // namespace

// ------------------------------------------------------------------ batches
// Independent problems grouped by velocity grid N: the cells of a group are
// concatenated in one state array and every collision kernel runs once over
// all of them; transport runs per problem on its segment of the array.
struct qb_batch_s {
  int precision = QB_F64;
  std::vector<qb_problem> probs;
  struct Group {
    qb_plan_s* plan = nullptr;
    std::vector<int> members;
    std::vector<Segment> segs;
    int total = 0;
    double* B = nullptr;  // [total][3]
  };
  std::vector<Group> groups;
  hipStream_t cap = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  std::vector<uintptr_t> key;
  size_t ws_used = 0;
  size_t bytes() const { return ws_used; }
  void drop_graph() {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    exec = nullptr;
    graph = nullptr;
    key.clear();
  }
  ~qb_batch_s() {
    (void)hipDeviceSynchronize();
    drop_graph();
    if (cap) (void)hipStreamDestroy(cap);
    for (Group& g : groups) delete g.plan;
  }
};

namespace {

template <typename T>
bool batch_enqueue(qb_batch_s* b, void* const* W, const double* const* B, double dt, int nsteps,
                   double* const* mom, hipStream_t s) {
  for (qb_batch_s::Group& g : b->groups) {
    qb_plan_s* pl = g.plan;
    const int N = pl->prob.N, ntot = g.total;
    const size_t per = (size_t)N * N, n = (size_t)ntot * per;
    T* cur = (T*)pl->st0;
    T* tmp = (T*)pl->st2;
    T* w1 = (T*)pl->st1;
    T* c = (T*)pl->cbuf;
    for (size_t k = 0; k < g.members.size(); ++k) {
      const int m = g.members[k];
      const Segment& sg = g.segs[k];
      if (!to_state<T, T>(pl, W[m], cur + (size_t)sg.offset * per, sg.Nx, s)) return false;
      hipLaunchKernelGGL(qb::k_copy_f64, dim3(blocks((size_t)sg.Nx * 3, 256)), dim3(256), 0, s, B ? B[m] : nullptr,
                         g.B + (size_t)sg.offset * 3, sg.Nx * 3);
    }
    // moments snapshot `snap` of every problem that asked for them, written
    // into its own array (component stride: the group's cell count)
    auto snap_moments = [&](const T* state, int snap) {
      if (!mom) return true;
      const int id = pl->begin(QB_K_MOMENTS, s);
      for (size_t k = 0; k < g.members.size(); ++k) {
        const int m = g.members[k];
        const Segment& sg = g.segs[k];
        if (!mom[m]) continue;
        hipLaunchKernelGGL((qb::k_moments<T>), dim3(sg.Nx), dim3(256), 0, s, state + (size_t)sg.offset * per,
                           mom[m] + (size_t)snap * sg.Nx * 7, ntot, N, pl->prob.L);
      }
      pl->end(id, s);
      return hip_ok(hipGetLastError(), "moments launch");
    };
    if (!snap_moments(cur, 0)) return false;
    auto half = [&](T*& a, T*& t) {
      const int id = pl->begin(QB_K_TRANSPORT, s);
      for (const Segment& sg : g.segs) transport_seg<T>(pl, a, t, 0.5 * dt, sg, ntot, s);
      pl->end(id, s);
      std::swap(a, t);
      return hip_ok(hipGetLastError(), "transport launch");
    };
    for (int it = 0; it < nsteps; ++it) {
      if (!half(cur, tmp)) return false;
      if (!collision_any<T>(pl, cur, c, ntot, s)) return false;
      int id = pl->begin(QB_K_HEUN, s);
      hipLaunchKernelGGL((qb::k_heun<T>), dim3(blocks(n, 256)), dim3(256), 0, s, cur, w1, c, g.B, (T)dt, ntot, N, 1);
      pl->end(id, s);
      if (!collision_any<T>(pl, w1, c, ntot, s)) return false;
      id = pl->begin(QB_K_HEUN, s);
      hipLaunchKernelGGL((qb::k_heun<T>), dim3(blocks(n, 256)), dim3(256), 0, s, cur, w1, c, g.B, (T)dt, ntot, N, 2);
      pl->end(id, s);
      if (!half(cur, tmp)) return false;
      if (!snap_moments(cur, it + 1)) return false;
    }
    for (size_t k = 0; k < g.members.size(); ++k) {
      const int m = g.members[k];
      const Segment& sg = g.segs[k];
      if (!from_state<T, T>(pl, cur + (size_t)sg.offset * per, W[m], sg.Nx, s)) return false;
    }
    if (!hip_ok(hipGetLastError(), "batch launch")) return false;
  }
  return true;
}

// One group of a batch: its plan over all of the group's cells (periodic
// placeholder walls), each member's wall tables and the group's field
// array, carved from the group plan's workspace.
template <typename T>
bool group_layout(qb_batch_s* b, qb_batch_s::Group& g) {
  qb_plan_s* pl = g.plan;
  if (!layout_plan<T>(pl)) return false;
  g.segs.clear();
  int off = 0;
  for (int m : g.members) {
    const qb_problem& p = b->probs[m];
    Segment sg{off, p.Nx, {}, {}, nullptr, nullptr, p.left.kind == QB_MAXWELL, p.right.kind == QB_MAXWELL};
    void* bcw = nullptr;
    if (!build_bc_for<T>(pl, p, sg.bl, sg.br, &bcw, &sg.flux)) return false;
    sg.bcw = bcw;
    g.segs.push_back(sg);
    off += p.Nx;
  }
  return pl->alloc((void**)&g.B, (size_t)g.total * 3 * sizeof(double));
}

qb_problem group_problem(const qb_batch_s* b, const qb_batch_s::Group& g) {
  qb_problem gp = b->probs[g.members[0]];
  gp.Nx = g.total;
  gp.left.kind = QB_PERIODIC;
  gp.right.kind = QB_PERIODIC;
  return gp;
}

// Lay out every group in [ws, ws + ws_bytes) (measuring when ws is null):
// group k's plan workspace starts at a 256-byte boundary after group k-1's.
qb_status batch_layout(qb_batch_s* b, void* ws, size_t ws_bytes) {
  const bool measure = ws == nullptr;
  size_t off = 0;
  for (qb_batch_s::Group& g : b->groups) {
    off = (off + 255) & ~(size_t)255;
    qb_plan_s* pl = new qb_plan_s();
    init_plan(pl, group_problem(b, g), 0);
    pl->ws.reset(measure ? nullptr : (char*)ws + off, measure ? 0 : (off < ws_bytes ? ws_bytes - off : 0), measure);
    g.plan = pl;
    const bool ok = b->precision == QB_F64 ? group_layout<double>(b, g) : group_layout<float>(b, g);
    if (!ok) return measure ? QB_EHIP : QB_EWORKSPACE;
    off += pl->ws.used;
  }
  b->ws_used = off;
  return QB_OK;
}

// Validate a batch description and group its problems by N.
qb_status batch_groups(const qb_problem* problems, int nprob, qb_batch_s* b) {
  const qb_problem& p0 = problems[0];
  for (int i = 0; i < nprob; ++i) {
    const qb_problem& p = problems[i];
    const qb_status st = validate(&p);
    if (st != QB_OK) return st;
    if (p.precision != p0.precision || p.J != p0.J || p.L != p0.L || p.R != p0.R) return QB_EINVAL;
  }
  b->precision = p0.precision;
  b->probs.assign(problems, problems + nprob);
  for (int i = 0; i < nprob; ++i) {
    const qb_problem& p = problems[i];
    qb_batch_s::Group* g = nullptr;
    for (auto& x : b->groups)
      if (b->probs[x.members[0]].N == p.N) g = &x;
    if (!g) {
      b->groups.emplace_back();
      g = &b->groups.back();
    } else if (b->probs[g->members[0]].M != p.M) {
      return QB_EINVAL;
    }
    g->members.push_back(i);
    g->total += p.Nx;
  }
  return QB_OK;
}

}  // namespace

// ------------------------------------------------------------------ static scratch
// Device memory of the library itself, for qb_collision_static: callers that
// cannot allocate (code under HIP graph capture, serving loops, harnesses
// that forbid allocation) get the collision's per-cell buffers from this
// array.  Each GPU the library runs on holds its own copy until the process
// ends.  Host code never names the array except to resolve its device
// address (per device, with that device current) through hipGetSymbolAddress.
constexpr size_t kStaticScratchBytes = (size_t)64 << 20;
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of this GPU's scratch array (resolved once per device);
// null after a failed HIP call (qb_last_error says which).
void* scratch_ptr() {
  int dev = -1;
  if (!hip_ok(hipGetDevice(&dev), "hipGetDevice")) return nullptr;
  if (dev < 0 || dev >= kMaxDevices) {
    set_error("device index beyond the scratch table");
    return nullptr;
  }
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    if (!hip_ok(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)), "hipGetSymbolAddress")) return nullptr;
    g_scratch_ptr[dev] = ptr;
  }
  return g_scratch_ptr[dev];
}

// Bytes of the static path's buffers for chunks of n cells: the collision
// buffers plus the state-sized input and output arrays of the chunk.
template <typename T>
size_t static_bytes(const qb_plan_s* pl, int n) {
  Arena a;
  a.reset(nullptr, 0, true);
  CollBufs b;
  void* x = nullptr;
  const size_t st = (size_t)4 * n * pl->prob.N * pl->prob.N * sizeof(T);
  carve_collision<T>(a, pl, n, b);
  a.take(&x, st);
  a.take(&x, st);
  return a.used;
}

// Largest chunk of at most `want` cells whose buffers fit the scratch
// array (0 if a single cell does not fit).
template <typename T>
int static_chunk(const qb_plan_s* pl, int want) {
  int lo = 0, hi = std::max(1, std::min(want, kChunkCells));
  while (lo < hi) {
    const int mid = (lo + hi + 1) / 2;
    if (static_bytes<T>(pl, mid) <= kStaticScratchBytes)
      lo = mid;
    else
      hi = mid - 1;
  }
  return lo;
}

// C[W] for ncells cells with every per-cell buffer in the scratch array:
// chunks of `chunk` cells, each converted to the Pauli layout, run through
// the same collision pipeline as qb_collision and converted back.  The
// plan's buffer pointers and cell count are switched to the scratch layout
// while the chunk's launches are enqueued and restored afterwards (the
// kernels take them by value at launch).
template <typename T>
qb_status do_collision_static(qb_plan_s* pl, void* base, const void* W, void* C, int ncells, int chunk,
                              hipStream_t s) {
  Arena a;
  a.reset(base, kStaticScratchBytes, false);
  CollBufs b;
  void *w = nullptr, *c = nullptr;
  const size_t per = (size_t)pl->prob.N * pl->prob.N;
  const size_t st = 4 * (size_t)chunk * per * sizeof(T);
  if (!carve_collision<T>(a, pl, chunk, b) || !a.take(&w, st) || !a.take(&c, st)) {
    set_error("static scratch exhausted");
    return QB_EWORKSPACE;
  }
  const CollBufs keep = get_bufs(pl);
  const int keep_nx = pl->prob.Nx, keep_wc = pl->wcells;
  set_bufs(pl, b);
  bool ok = true;
  for (int c0 = 0; c0 < ncells && ok; c0 += chunk) {
    const int n = std::min(chunk, ncells - c0);
    // state arrays of the chunk hold n cells per Pauli component
    pl->prob.Nx = n;
    pl->wcells = n;
    const T* Wc = (const T*)W + (size_t)c0 * per * 8;
    T* Cc = (T*)C + (size_t)c0 * per * 8;
    hipLaunchKernelGGL((qb::k_api_to_state<T, T>), dim3(blocks(n * per, 256)), dim3(256), 0, s, Wc, (T*)w, n,
                       pl->prob.N, n);
    ok = hip_ok(hipGetLastError(), "layout launch") && collision_chunk<T>(pl, (const T*)w, (T*)c, n, 0, s);
    if (ok) {
      hipLaunchKernelGGL((qb::k_state_to_api<T, T>), dim3(blocks(n * per, 256)), dim3(256), 0, s, (const T*)c, Cc, n,
                         pl->prob.N, n);
      ok = hip_ok(hipGetLastError(), "layout launch");
    }
  }
  set_bufs(pl, keep);
  pl->prob.Nx = keep_nx;
  pl->wcells = keep_wc;
  return ok ? QB_OK : QB_EHIP;
}

}  // namespace

// ------------------------------------------------------------------ C ABI
extern "C" {

size_t qb_workspace_bytes(const qb_problem* problem, int32_t max_cells) {
  if (validate(problem) != QB_OK || max_cells < 0) return 0;
  return plan_workspace_bytes(*problem, max_cells);
}

qb_status qb_plan_create(const qb_problem* problem, int32_t max_cells, void* workspace, size_t ws_bytes,
                         qb_plan* out) {
  if (!out) return QB_EINVAL;
  *out = nullptr;
  qb_status st = validate(problem);
  if (st != QB_OK) return st;
  if (max_cells < 0 || !workspace) return QB_EINVAL;
  if (ws_bytes < plan_workspace_bytes(*problem, max_cells)) return QB_EWORKSPACE;
  qb_plan_s* pl = create_plan(*problem, max_cells, workspace, ws_bytes);
  if (!pl) return QB_EHIP;
  // set-up of qb_collision_static on this device
  if (!scratch_ptr()) {
    delete pl;
    return QB_EHIP;
  }
  *out = pl;
  return QB_OK;
}

qb_status qb_plan_destroy(qb_plan plan) {
  if (!plan) return QB_EINVAL;
  (void)hipDeviceSynchronize();
  delete plan;
  return QB_OK;
}

size_t qb_plan_bytes(qb_plan plan) { return plan ? plan->bytes() : 0; }

int32_t qb_plan_chunk_cells(qb_plan plan) { return plan ? plan->wcells : 0; }

qb_status qb_collision(qb_plan plan, const void* W, void* C, int32_t ncells, void* stream) {
  if (!plan || !W || !C || W == C) return QB_EINVAL;
  if (ncells < 1) return QB_EINVAL;
  if (ncells > plan->prob.Nx) return QB_EWORKSPACE;
  hipStream_t s = (hipStream_t)stream;
  if (plan->prob.precision == QB_F64) return do_collision<double>(plan, W, C, ncells, s);
  return do_collision<float>(plan, W, C, ncells, s);
}

size_t qb_collision_static_bytes(void) { return kStaticScratchBytes; }

qb_status qb_collision_static(qb_plan plan, const void* W, void* C, int32_t ncells, void* stream) {
  if (!plan || !W || !C || W == C) return QB_EINVAL;
  if (ncells < 1) return QB_EINVAL;
  if (ncells > plan->prob.Nx) return QB_EWORKSPACE;
  const bool f64 = plan->prob.precision == QB_F64;
  const int chunk = f64 ? static_chunk<double>(plan, ncells) : static_chunk<float>(plan, ncells);
  if (chunk < 1) {
    set_error("one cell's collision buffers exceed the static scratch of qb_collision_static");
    return QB_EWORKSPACE;
  }
  void* base = scratch_ptr();
  if (!base) return QB_EHIP;
  hipStream_t s = (hipStream_t)stream;
  return f64 ? do_collision_static<double>(plan, base, W, C, ncells, chunk, s)
             : do_collision_static<float>(plan, base, W, C, ncells, chunk, s);
}

static qb_status check_cfl(qb_plan plan, double dt) {
  const qb_problem& p = plan->prob;
  if (!(dt >= 0.0) || !std::isfinite(dt)) return QB_EINVAL;
  const double vmax = p.L;  // |v_x| <= L on the grid (row v_x = -L)
  if (dt * vmax * p.Nx > 1.0 + 1e-12) return QB_ECFL;
  return QB_OK;
}

qb_status qb_transport_step(qb_plan plan, void* W, double dt, void* stream) {
  if (!plan || !W) return QB_EINVAL;
  qb_status st = check_cfl(plan, dt);
  if (st != QB_OK) return st;
  hipStream_t s = (hipStream_t)stream;
  if (plan->prob.precision == QB_F64) return do_transport<double>(plan, W, dt, s);
  return do_transport<float>(plan, W, dt, s);
}

qb_status qb_step(qb_plan plan, void* W, const double* B, double dt, int32_t nsteps, double* moments_out,
                  void* stream) {
  if (!plan || !W || nsteps < 0) return QB_EINVAL;
  qb_status st = check_cfl(plan, 0.5 * dt);
  if (st != QB_OK) return st;
  hipStream_t s = (hipStream_t)stream;
  if (plan->prob.precision == QB_F64) return do_step<double>(plan, W, B, dt, nsteps, moments_out, nullptr, s);
  return do_step<float>(plan, W, B, dt, nsteps, moments_out, nullptr, s);
}

qb_status qb_step_fluxes(qb_plan plan, void* W, const double* B, double dt, int32_t nsteps, double* moments_out,
                         double* inflow, void* stream) {
  if (!plan || !W || !inflow || nsteps < 0) return QB_EINVAL;
  qb_status st = check_cfl(plan, 0.5 * dt);
  if (st != QB_OK) return st;
  hipStream_t s = (hipStream_t)stream;
  if (plan->prob.precision == QB_F64) return do_step<double>(plan, W, B, dt, nsteps, moments_out, nullptr, s, inflow);
  return do_step<float>(plan, W, B, dt, nsteps, moments_out, nullptr, s, inflow);
}

size_t qb_adjoint_workspace_bytes(qb_plan plan) { return plan ? adjoint_workspace_bytes(plan) : 0; }

qb_status qb_plan_enable_adjoint(qb_plan plan, void* workspace, size_t ws_bytes) {
  if (!plan) return QB_EINVAL;
  if (plan->adjoint) return QB_OK;
  if (!workspace) return QB_EINVAL;
  if (ws_bytes < adjoint_workspace_bytes(plan)) return QB_EWORKSPACE;
  plan->adj.reset(workspace, ws_bytes, false);
  const bool ok = plan->prob.precision == QB_F64 ? build_adjoint<double>(plan) : build_adjoint<float>(plan);
  if (!ok) return QB_EWORKSPACE;
  plan->adjoint = true;
  return QB_OK;
}

size_t qb_trace_bytes(qb_plan plan) {
  if (!plan) return 0;
  const qb_problem& p = plan->prob;
  const size_t b = p.precision == QB_F64 ? sizeof(double) : sizeof(float);
  return (size_t)3 * 4 * p.Nx * p.N * p.N * b;
}

qb_status qb_step_trace(qb_plan plan, void* W, const double* B, double dt, int32_t nsteps, void* trace,
                        void* stream) {
  if (!plan || !W || !trace || nsteps < 0) return QB_EINVAL;
  if (plan->limiter != QB_LIMITER_MINMOD || plan->field_mode != QB_FIELD_HEUN) return QB_ENOTSUP;
  qb_status st = check_cfl(plan, 0.5 * dt);
  if (st != QB_OK) return st;
  hipStream_t s = (hipStream_t)stream;
  if (plan->prob.precision == QB_F64) return do_step<double>(plan, W, B, dt, nsteps, nullptr, (double*)trace, s);
  return do_step<float>(plan, W, B, dt, nsteps, nullptr, (float*)trace, s);
}

qb_status qb_collision_vjp(qb_plan plan, const void* W, const void* lam, void* G, int32_t ncells, void* stream) {
  if (!plan || !W || !lam || !G || ncells < 1) return QB_EINVAL;
  if (ncells > plan->prob.Nx || !plan->adjoint) return QB_EWORKSPACE;
  if (plan->term_sel != QB_TERMS_ALL) return QB_ENOTSUP;
  hipStream_t s = (hipStream_t)stream;
  if (plan->prob.precision == QB_F64) return do_collision_vjp<double>(plan, W, lam, G, ncells, s);
  return do_collision_vjp<float>(plan, W, lam, G, ncells, s);
}

qb_status qb_transport_vjp(qb_plan plan, const void* W, double dt, const void* lam, void* G, void* stream) {
  if (!plan || !W || !lam || !G) return QB_EINVAL;
  if (!plan->adjoint) return QB_EWORKSPACE;
  if (plan->limiter != QB_LIMITER_MINMOD) return QB_ENOTSUP;
  qb_status st = check_cfl(plan, dt);
  if (st != QB_OK) return st;
  hipStream_t s = (hipStream_t)stream;
  if (plan->prob.precision == QB_F64) return do_transport_vjp<double>(plan, W, dt, lam, G, s);
  return do_transport_vjp<float>(plan, W, dt, lam, G, s);
}

qb_status qb_adjoint_step(qb_plan plan, const void* W, const void* record, const double* B, double dt,
                          const void* lam_next, void* lam, double* gB, void* stream) {
  if (!plan || (!W && !record) || !lam_next || !lam) return QB_EINVAL;
  if (!plan->adjoint) return QB_EWORKSPACE;
  if (plan->term_sel != QB_TERMS_ALL) return QB_ENOTSUP;
  if (plan->limiter != QB_LIMITER_MINMOD || plan->field_mode != QB_FIELD_HEUN) return QB_ENOTSUP;
  qb_status st = check_cfl(plan, 0.5 * dt);
  if (st != QB_OK) return st;
  hipStream_t s = (hipStream_t)stream;
  if (plan->prob.precision == QB_F64) return do_adjoint_step<double>(plan, W, record, B, dt, lam_next, lam, gB, s);
  return do_adjoint_step<float>(plan, W, record, B, dt, lam_next, lam, gB, s);
}

qb_status qb_moments(qb_plan plan, const void* W, double* mom, void* stream) {
  if (!plan || !W || !mom) return QB_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  if (plan->prob.precision == QB_F64) return do_moments<double>(plan, W, mom, s);
  return do_moments<float>(plan, W, mom, s);
}

qb_status qb_diagnostics(qb_plan plan, const void* W, const void* C, const qb_fd* global, double* out,
                         void* stream) {
  if (!plan || !W || !out) return QB_EINVAL;
  qb::FdGlobal g{};
  if (global) {
    // Bloch vector of the spin-up projector: first column (a, b) of U
    const double ar = global->U_re[0], ai = global->U_im[0], br = global->U_re[2], bi = global->U_im[2];
    const double nn = ar * ar + ai * ai + br * br + bi * bi;
    if (!(global->inv_kT > 0.0) || !std::isfinite(global->inv_kT) || !std::isfinite(global->mu_up) ||
        !std::isfinite(global->mu_down) || !(nn > 0.0) || !std::isfinite(nn))
      return QB_EINVAL;
    g.inv_kT = global->inv_kT;
    g.mu_up = global->mu_up;
    g.mu_down = global->mu_down;
    g.n[0] = 2.0 * (ar * br + ai * bi) / nn;  // 2 Re(conj(a) b)
    g.n[1] = 2.0 * (ar * bi - ai * br) / nn;  // 2 Im(conj(a) b)
    g.n[2] = (ar * ar + ai * ai - br * br - bi * bi) / nn;
    g.valid = 1;
  }
  hipStream_t s = (hipStream_t)stream;
  if (plan->prob.precision == QB_F64) return do_diagnostics<double>(plan, W, C, g, out, s);
  return do_diagnostics<float>(plan, W, C, g, out, s);
}

const char* qb_strerror(qb_status status) {
  switch (status) {
    case QB_OK: return "ok";
    case QB_EINVAL: return "invalid argument";
    case QB_ENOTSUP: return "unsupported problem size (N must be 16, 32 or 64; J even)";
    case QB_ECFL: return "CFL condition violated: dt max|v_x| / dx > 1";
    case QB_EWORKSPACE: return "more cells than the plan holds";
    case QB_EHIP: return "HIP runtime error";
  }
  return "unknown status";
}

const char* qb_last_error(void) { return g_last_error.c_str(); }

qb_status qb_profile(qb_plan plan, int32_t enable) {
  if (!plan) return QB_EINVAL;
  plan->profiling = enable != 0;
  return QB_OK;
}

qb_status qb_profile_read(qb_plan plan, int32_t kernel, double* total_ms, int64_t* launches) {
  if (!plan || !total_ms || !launches || kernel < 0 || kernel >= QB_K_COUNT) return QB_EINVAL;
  double ms = 0.0;
  int64_t n = 0;
  std::vector<qb_plan_s::Rec> keep;
  for (auto& r : plan->recs) {
    if (r.kernel != kernel) {
      keep.push_back(r);
      continue;
    }
    if (!hip_ok(hipEventSynchronize(r.b), "hipEventSynchronize")) return QB_EHIP;
    float e = 0.f;
    if (!hip_ok(hipEventElapsedTime(&e, r.a, r.b), "hipEventElapsedTime")) return QB_EHIP;
    ms += e;
    ++n;
    plan->pool.push_back(r.a);
    plan->pool.push_back(r.b);
  }
  plan->recs.swap(keep);
  *total_ms = ms;
  *launches = n;
  return QB_OK;
}

qb_status qb_plan_set_tile(qb_plan plan, int32_t E) {
  if (!plan) return QB_EINVAL;
  const std::vector<int> c = tile_candidates(plan->P);
  if (std::find(c.begin(), c.end(), (int)E) == c.end()) return QB_ENOTSUP;
  const bool ok = plan->prob.precision == QB_F64 ? select_tile<double>(plan, E) : select_tile<float>(plan, E);
  return ok ? QB_OK : QB_EHIP;
}

qb_status qb_plan_set_scheme(qb_plan plan, int32_t limiter, int32_t field) {
  if (!plan || limiter < QB_LIMITER_MINMOD || limiter > QB_LIMITER_VAN_LEER || field < QB_FIELD_HEUN ||
      field > QB_FIELD_ROTATION)
    return QB_EINVAL;
  plan->limiter = limiter;
  plan->field_mode = field;
  return QB_OK;
}

qb_status qb_plan_set_terms(qb_plan plan, int32_t terms) {
  if (!plan || terms < QB_TERMS_CONSERVATIVE || terms > QB_TERMS_ALL) return QB_EINVAL;
  plan->term_sel = terms;
  return QB_OK;
}

qb_status qb_plan_set_pairing(qb_plan plan, int32_t paired) {
  if (!plan || paired < 0 || paired > 1) return QB_EINVAL;
  plan->i3_pair = paired == 1;
  return QB_OK;
}

qb_status qb_plan_set_adjoint_tile(qb_plan plan, int32_t E) {
  if (!plan) return QB_EINVAL;
  if (E != 0) {
    const std::vector<int> c = tile_candidates(plan->P);
    if (std::find(c.begin(), c.end(), (int)E) == c.end()) return QB_ENOTSUP;
  }
  const bool ok = plan->prob.precision == QB_F64 ? select_vjp_tile<double>(plan, E) : select_vjp_tile<float>(plan, E);
  return ok ? QB_OK : QB_EHIP;
}

qb_status qb_plan_set_persistent(qb_plan plan, int32_t persistent) {
  if (!plan || persistent < 0 || persistent > 1) return QB_EINVAL;
  plan->persistent = persistent == 1;
  return QB_OK;
}

qb_status qb_plan_set_adjoint_variant(qb_plan plan, int32_t variant) {
  if (!plan || variant < 0 || variant > 1) return QB_EINVAL;
  plan->vjp_variant = variant;
  return QB_OK;
}

qb_status qb_plan_config(qb_plan plan, int32_t* tile, int32_t* adjoint_variant, int32_t* paired_nodes,
                         int32_t* adjoint_tile, int32_t* persistent) {
  if (!plan) return QB_EINVAL;
  if (persistent) *persistent = plan->persistent ? 1 : 0;
  if (tile) *tile = plan->E;
  if (adjoint_tile) *adjoint_tile = plan->tabs[plan->vjp_tab].E;
  if (adjoint_variant) *adjoint_variant = plan->vjp_variant;
  if (paired_nodes) *paired_nodes = plan->i3_pair ? 1 : 0;
  return QB_OK;
}

qb_status qb_plan_tune(qb_plan plan, int32_t ncells, int32_t* tile, void* stream) {
  if (!plan || ncells < 1) return QB_EINVAL;
  if (ncells > plan->prob.Nx) return QB_EWORKSPACE;
  int chosen = 0;
  hipStream_t s = (hipStream_t)stream;
  const qb_status st = plan->prob.precision == QB_F64 ? do_tune<double>(plan, ncells, &chosen, s)
                                                      : do_tune<float>(plan, ncells, &chosen, s);
  if (st == QB_OK && tile) *tile = chosen;
  return st;
}

size_t qb_batch_workspace_bytes(const qb_problem* problems, int32_t nprob) {
  if (!problems || nprob < 1) return 0;
  qb_batch_s b;
  if (batch_groups(problems, nprob, &b) != QB_OK || batch_layout(&b, nullptr, 0) != QB_OK) return 0;
  return b.ws_used;
}

qb_status qb_batch_create(const qb_problem* problems, int32_t nprob, void* workspace, size_t ws_bytes,
                          qb_batch* out) {
  if (!out || !problems || nprob < 1) return QB_EINVAL;
  *out = nullptr;
  qb_batch_s* b = new qb_batch_s();
  qb_status st = batch_groups(problems, nprob, b);
  if (st == QB_OK && !workspace) st = QB_EINVAL;
  if (st == QB_OK && ws_bytes < qb_batch_workspace_bytes(problems, nprob)) st = QB_EWORKSPACE;
  if (st == QB_OK) st = batch_layout(b, workspace, ws_bytes);
  if (st == QB_OK && !hip_ok(hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking), "hipStreamCreate"))
    st = QB_EHIP;
  if (st != QB_OK) {
    delete b;
    return st;
  }
  *out = b;
  return QB_OK;
}

qb_status qb_batch_destroy(qb_batch batch) {
  if (!batch) return QB_EINVAL;
  delete batch;
  return QB_OK;
}

size_t qb_batch_bytes(qb_batch batch) { return batch ? batch->bytes() : 0; }

qb_status qb_batch_tune(qb_batch batch, void* stream) {
  if (!batch) return QB_EINVAL;
  for (auto& g : batch->groups) {
    const int n = std::min(g.total, g.plan->wcells);
    const qb_status st = qb_plan_tune(g.plan, n, nullptr, stream);
    if (st != QB_OK) return st;
  }
  batch->drop_graph();  // recorded launches refer to the previous tiles
  return QB_OK;
}

qb_status qb_batch_set_persistent(qb_batch batch, int32_t persistent) {
  if (!batch || persistent < 0 || persistent > 1) return QB_EINVAL;
  for (auto& g : batch->groups) g.plan->persistent = persistent == 1;
  batch->drop_graph();  // recorded launches use the previous shape
  return QB_OK;
}

qb_status qb_batch_step(qb_batch batch, void* const* W, const double* const* B, double dt, int32_t nsteps,
                        double* const* moments, int32_t flags, void* stream) {
  if (!batch || !W || nsteps < 0 || !(dt >= 0.0) || !std::isfinite(dt)) return QB_EINVAL;
  const int np = (int)batch->probs.size();
  for (int m = 0; m < np; ++m) {
    const qb_problem& p = batch->probs[m];
    if (!W[m]) return QB_EINVAL;
    if (0.5 * dt * p.L * p.Nx > 1.0 + 1e-12) return QB_ECFL;
  }
  hipStream_t s = (hipStream_t)stream;
  auto run = [&](hipStream_t q) {
    return batch->precision == QB_F64 ? batch_enqueue<double>(batch, W, B, dt, nsteps, moments, q)
                                      : batch_enqueue<float>(batch, W, B, dt, nsteps, moments, q);
  };
  if (!(flags & QB_BATCH_GRAPH)) return run(s) ? QB_OK : QB_EHIP;
  // graph replay: one recorded launch sequence per argument set
  std::vector<uintptr_t> key;
  for (int m = 0; m < np; ++m) {
    key.push_back((uintptr_t)W[m]);
    key.push_back((uintptr_t)(B ? B[m] : nullptr));
    key.push_back((uintptr_t)(moments ? moments[m] : nullptr));
  }
  uint64_t dbits;
  std::memcpy(&dbits, &dt, sizeof dbits);
  key.push_back((uintptr_t)dbits);
  key.push_back((uintptr_t)nsteps);
  if (!batch->exec || key != batch->key) {
    batch->drop_graph();
    std::vector<bool> prof;
    for (auto& g : batch->groups) {
      prof.push_back(g.plan->profiling);
      g.plan->profiling = false;
    }
    if (!hip_ok(hipStreamBeginCapture(batch->cap, hipStreamCaptureModeThreadLocal), "hipStreamBeginCapture"))
      return QB_EHIP;
    const bool ok = run(batch->cap);
    hipGraph_t graph = nullptr;
    const bool ended = hip_ok(hipStreamEndCapture(batch->cap, &graph), "hipStreamEndCapture");
    for (size_t i = 0; i < batch->groups.size(); ++i) batch->groups[i].plan->profiling = prof[i];
    if (!ok || !ended) {
      if (graph) (void)hipGraphDestroy(graph);
      return QB_EHIP;
    }
    batch->graph = graph;
    if (!hip_ok(hipGraphInstantiate(&batch->exec, graph, nullptr, nullptr, 0), "hipGraphInstantiate")) {
      batch->drop_graph();
      return QB_EHIP;
    }
    batch->key = key;
  }
  return hip_ok(hipGraphLaunch(batch->exec, s), "hipGraphLaunch") ? QB_OK : QB_EHIP;
}

int32_t qb_version(void) { return 310; }

}  // extern "C"
