// Internal host interface shared by qb_lib.hip and the per-tile
// compilation units: the plan object, launch helpers and the collision
// pipelines (forward and reverse) instantiated for every tile shape.
#pragma once
#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "qb.h"
#include "qb_adjoint.hpp"
#include "qb_kernels.hpp"

using qb::DevPlan;

// Records the text of a failed HIP call for qb_last_error(); true on success.
bool hip_ok(hipError_t e, const char* what);
// Records a message for qb_last_error().
void set_error(const char* what);

// Workgroups of `threads` threads of kernel `kern` resident on the current
// device at once (occupancy x compute units), rounded down to a multiple of
// 8 (one per XCD, so a grid stride keeps its XCD); at least 8.
int persistent_grid(const void* kern, int threads);

// Bump allocator over caller-owned device memory: the library never
// allocates device memory itself.  In measuring mode it only adds up the
// aligned sizes (the pointers stay null), which is how the workspace size
// of a problem is computed from the same layout code that carves it.
struct Arena {
  char* base = nullptr;
  size_t cap = 0, used = 0;
  bool measure = true;
  void reset(void* b, size_t c, bool m) {
    base = (char*)b;
    cap = c;
    used = 0;
    measure = m;
  }
  bool take(void** p, size_t n) {
    const size_t off = (used + 255) & ~(size_t)255;
    if (!measure && off + n > cap) return false;
    *p = measure ? nullptr : base + off;
    used = off + n;
    return true;
  }
};

inline int blocks(size_t n, int b) { return (int)((n + b - 1) / b); }

struct qb_plan_s {
  qb_problem prob;
  Arena ws;   // the plan's workspace (tables, walls, collision and state buffers)
  Arena adj;  // the reverse-mode workspace (qb_plan_enable_adjoint)
  int P, E, NT, TPR;
  int wcells;  // cells per collision launch (the workspace holds this many)
  bool i3_pair = true;  // I_3 kernel pairs the Gauss-Legendre nodes (tuned; default per tile)
  int vjp_variant = 0;  // I_3 adjoint: 0 row w_bar in memory, 1 in registers (tuned)
  int vjp_E = 0;        // tile shape of the reverse-mode pipeline (tuned; 0: the forward tile)
  int vjp_tab = 0;      // its table set
  int term_sel = 3;     // collision terms assembled: 1 C_c, 2 C_d, 3 both
  int limiter = 0;      // transport slope limiter: 0 minmod, 1 superbee, 2 MC, 3 van Leer
  int field_mode = 0;   // field term: 0 inside the Heun step, 1 exact rotation split around it
  bool persistent = false;  // collision kernels grid-stride over their tasks from a resident-sized grid
  // quadrature tables in the FFT engine's element order, one set per tile
  // shape E (elements per thread) that has been selected on this plan
  struct TabSet {
    int E = 0;
    bool built = false;
    void *tw = nullptr, *phip = nullptr, *Kt = nullptr, *psi = nullptr, *psip = nullptr, *psiw = nullptr,
         *psips = nullptr, *negk = nullptr;
  };
  std::vector<TabSet> tabs;
  int cur_tab = 0;
  void *phx, *phy, *wm;  // natural order, independent of the tile
  void *spec, *wP, *terms, *acc, *i3s = nullptr, *i3o, *i3sum, *i3p, *i3ps;
  void *st0, *st1, *st2, *cbuf, *bcw;
  double* flux;
  // adjoint workspace (qb_plan_enable_adjoint)
  bool adjoint = false;
  void *lamP = nullptr, *acot = nullptr, *gspec = nullptr, *gf0 = nullptr, *i3g = nullptr,
       *i3sb = nullptr, *gsum = nullptr, *i3t = nullptr, *lamh = nullptr;
  void *fwa = nullptr;
  void *wn = nullptr, *wa = nullptr, *w1 = nullptr, *wb = nullptr, *lb = nullptr, *ls = nullptr, *la = nullptr,
       *cg = nullptr, *g0 = nullptr, *ext = nullptr;
  double* lflux = nullptr;
  qb::BcDev bl, br;
  // kernel timing
  bool profiling = false;
  struct Rec {
    int kernel;
    hipEvent_t a, b;
  };
  std::vector<Rec> recs;
  std::vector<hipEvent_t> pool;

  bool measuring() const { return ws.measure; }
  // carve n bytes of the plan workspace (false once it is exhausted)
  bool alloc(void** p, size_t n) {
    if (ws.take(p, n)) return true;
    set_error("plan workspace exhausted");
    return false;
  }
  bool alloc_adj(void** p, size_t n) {
    if (adj.take(p, n)) return true;
    set_error("adjoint workspace exhausted");
    return false;
  }
  size_t bytes() const { return ws.used + (adjoint ? adj.used : 0); }
  ~qb_plan_s() {
    for (auto& r : recs) {
      (void)hipEventDestroy(r.a);
      (void)hipEventDestroy(r.b);
    }
    for (hipEvent_t e : pool) (void)hipEventDestroy(e);
  }
  hipEvent_t event() {
    if (!pool.empty()) {
      hipEvent_t e = pool.back();
      pool.pop_back();
      return e;
    }
    hipEvent_t e = nullptr;
    (void)hipEventCreate(&e);
    return e;
  }
  // bracket one launch: call begin() before and end() after the launch
  int begin(int kernel, hipStream_t s) {
    if (!profiling) return -1;
    Rec r{kernel, event(), event()};
    (void)hipEventRecord(r.a, s);
    recs.push_back(r);
    return (int)recs.size() - 1;
  }
  void end(int id, hipStream_t s) {
    if (id >= 0) (void)hipEventRecord(recs[id].b, s);
  }
};


// Device view of the plan with the table set `tab` (the forward pipeline
// uses cur_tab, the reverse-mode pipeline vjp_tab).
template <typename T>
inline DevPlan<T> devplan(qb_plan_s* pl, int tab) {
  DevPlan<T> d;
  d.Nx = pl->prob.Nx;
  d.N = pl->prob.N;
  d.J = pl->prob.J;
  d.M = pl->prob.M;
  d.P = pl->P;
  d.L = (T)pl->prob.L;
  d.wc = (pl->term_sel & 1) ? (T)1 : (T)0;
  d.wd = (pl->term_sel & 2) ? (T)1 : (T)0;
  const qb_plan_s::TabSet& ts = pl->tabs[tab];
  d.tw = (const T*)ts.tw;
  d.phip = (const T*)ts.phip;
  d.Kt = (const T*)ts.Kt;
  d.psi = (const T*)ts.psi;
  d.psip = (const T*)ts.psip;
  d.psiw = (const T*)ts.psiw;
  d.psips = (const T*)ts.psips;
  d.negk = (const unsigned*)ts.negk;
  d.phx = (const T*)pl->phx;
  d.phy = (const T*)pl->phy;
  d.wm = (const T*)pl->wm;
  d.spec = (T*)pl->spec;
  d.wP = (T*)pl->wP;
  d.terms = (T*)pl->terms;
  d.acc = (T*)pl->acc;
  d.i3s = (T*)pl->i3s;
  d.i3o = (T*)pl->i3o;
  d.i3sum = (T*)pl->i3sum;
  d.i3p = (T*)pl->i3p;
  d.i3ps = (T*)pl->i3ps;
  d.lamP = (T*)pl->lamP;
  d.acot = (T*)pl->acot;
  d.gspec = (T*)pl->gspec;
  d.gf0 = (T*)pl->gf0;
  d.i3g = (T*)pl->i3g;
  d.i3sb = (T*)pl->i3sb;
  d.gsum = (T*)pl->gsum;
  d.fwa = (T*)pl->fwa;
  d.i3t = (T*)pl->i3t;
  d.lamh = (T*)pl->lamh;
  return d;
}


// C[w] for the cells [cell0, cell0 + ncells) of the Pauli state arrays w, c
// ([4][Nx][N][N]); ncells <= wcells, the workspace holds the chunk's cells
// from index 0.  Defined in qb_pipelines.hpp.
template <typename T, int P, int E>
bool collision_pipeline(qb_plan_s* pl, const T* w, T* c, int ncells, int cell0, hipStream_t s);

// out = C'(w)^T lam for the same cells (Pauli gradients).
template <typename T, int P, int E>
bool collision_vjp_pipeline(qb_plan_s* pl, const T* w, const T* lam, T* out, int ncells, int cell0,
                            hipStream_t s);
