// C ABI of the MI355X hot path: plan, workspace layout, forward / misfit /
// adjoint-gradient step loops.  See include/pmlfwi.h for the contract.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <mutex>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "pmlfwi.h"
#include <cmath>
#include <type_traits>

#include "kernels.h"
#include "regularize.h"
#include "mfma.h"
#include "convnet.h"

using namespace pmlfwi;

// Message of the last failed fwi_plan_create on this thread (no plan to hold it).
static thread_local std::string g_plan_err;

namespace {
// ---------------------------------------------------------------- checkpoint schedules
// With checkpoint spacing k the N steps fall into nseg segments; the adjoint
// reverses them last to first, recomputing each from the full state at its
// start (kept in a checkpoint slot) with the stage stores on.
//  * slots = 0: the forward keeps the state at every segment start.
//  * slots = c > 0: binomial checkpointing over the segments with c slots
//    (Griewank's "revolve" schedules, Griewank and Walther, ACM TOMS 26,
//    2000): reversing l segments from a held state with s free slots, advance
//    m segments, keep the state there, reverse the right part with s - 1
//    slots, then the left part with s.  The least total number of segment
//    advances has a closed form (revolve_cost); the split m is the first
//    that attains it.  The forward sweep already performs the first chain of
//    advances and keeps those states, so the adjoint starts at the last
//    segment.
enum ActKind { ACT_LOAD = 0, ACT_ADVANCE = 1, ACT_SAVE = 2, ACT_REVERSE = 3 };
struct Act {
  int kind, a, b;   // LOAD slot a (-1: the state at rest); ADVANCE segments a -> b;
                    // SAVE slot a; REVERSE segment a
};

// C(S + t, S), saturating above `cap`.
long long binom_capped(int S, long long t, long long cap) {
  long double b = 1.0L;
  for (long long i = 1; i <= t; ++i) {
    b = b * (long double)(S + i) / (long double)i;
    if (b > (long double)cap) return cap + 1;
  }
  return (long long)(b + 0.5L);
}

// Least number of segment advances that reverse l segments from a held state
// with s free slots: 0 for l <= 1, l (l - 1) / 2 with no slot, else with
// S = s + 1 snapshots and t the least integer with C(S + t, S) >= l,
// t l - C(S + t, S + 1).
long long revolve_cost(long long l, int s) {
  if (l <= 1) return 0;
  if (s == 0) return l * (l - 1) / 2;
  const int S = s + 1;
  long long t = 0;
  while (binom_capped(S, t, l) < l) ++t;
  return t * l - binom_capped(S + 1, t - 1, (long long)1 << 62);
}

int revolve_split(int l, int s) {
  const long long best = revolve_cost(l, s);
  for (int m = 1; m < l; ++m)
    if (m + revolve_cost(l - m, s - 1) + revolve_cost(m, s) == best) return m;
  return 1;
}

void revolve_gen(int first, int last, int s, int src, bool pre, int slots, std::vector<Act>& out,
                 std::vector<int>& fwd_slot) {
  const int l = last - first;
  if (l == 1) {
    out.push_back({ACT_LOAD, src, 0});
    out.push_back({ACT_REVERSE, first, 0});
    return;
  }
  if (s == 0) {
    for (int j = l - 1; j >= 0; --j) {
      out.push_back({ACT_LOAD, src, 0});
      if (j > 0) out.push_back({ACT_ADVANCE, first, first + j});
      out.push_back({ACT_REVERSE, first + j, 0});
    }
    return;
  }
  const int m = revolve_split(l, s);
  const int slot = slots - s;
  if (pre) {
    fwd_slot[first + m] = slot;
  } else {
    out.push_back({ACT_LOAD, src, 0});
    out.push_back({ACT_ADVANCE, first, first + m});
    out.push_back({ACT_SAVE, slot, 0});
  }
  revolve_gen(first + m, last, s - 1, slot, pre, slots, out, fwd_slot);
  revolve_gen(first, first + m, s, src, false, slots, out, fwd_slot);
}

struct Schedule {
  std::vector<Act> acts;       // adjoint actions
  std::vector<int> fwd_slot;   // per segment start: slot the forward keeps it in, or -1
  int nseg = 0, slots = 0;     // slots actually used
  long long advances = 0;      // segment advances of forward chain + adjoint
  long long adjoint_steps = 0; // forward steps the adjoint recomputes
};

Schedule make_schedule(const fwi_problem& P) {
  Schedule S;
  const int k = P.ckpt_every;
  if (k <= 0) return S;
  S.nseg = (P.nsteps + k - 1) / k;
  S.fwd_slot.assign(S.nseg, -1);
  if (P.ckpt_slots == 0 || P.ckpt_slots >= S.nseg - 1) {
    // a slot for every segment start (segment 0: the state at rest)
    S.slots = S.nseg;
    for (int g = 0; g < S.nseg; ++g) S.fwd_slot[g] = g;
    for (int g = S.nseg - 1; g >= 0; --g) {
      S.acts.push_back({ACT_LOAD, g, 0});
      S.acts.push_back({ACT_REVERSE, g, 0});
    }
  } else {
    S.slots = P.ckpt_slots;
    revolve_gen(0, S.nseg, P.ckpt_slots, -1, true, P.ckpt_slots, S.acts, S.fwd_slot);
  }
  auto seg_len = [&](int g) { return std::min(P.nsteps, (g + 1) * k) - g * k; };
  long long chain = 0;
  for (int g = 1; g < S.nseg; ++g)
    if (S.fwd_slot[g] >= 0) chain = g;
  S.advances = chain;
  for (const Act& a : S.acts) {
    if (a.kind == ACT_ADVANCE) {
      S.advances += a.b - a.a;
      for (int g = a.a; g < a.b; ++g) S.adjoint_steps += seg_len(g);
    } else if (a.kind == ACT_REVERSE) {
      S.adjoint_steps += seg_len(a.a);
    }
  }
  return S;
}

}  // namespace

struct fwi_plan {
  fwi_problem prob;
  Geo g;
  int nsrc, nrec;
  std::vector<Tile> tiles_int, tiles_pml;
  Tile* d_tiles_int = nullptr;
  Tile* d_tiles_pml = nullptr;
  int32_t* d_src = nullptr;
  double* d_dir = nullptr;
  int32_t* d_rec = nullptr;
  // general nodal loads (fwi_plan_set_loads): entry e adds
  // load_vec[e] * wavelet[load_src[e]][k] at node load_node[e]; replaces the
  // point loads of fwi_plan_create when nload > 0
  int nload = 0;
  int32_t* d_load_src = nullptr;
  int32_t* d_load_node = nullptr;
  double* d_load_vec = nullptr;
  std::vector<double> tab;           // per-axis PML profile and 1D mass factors
  std::vector<int> fo;               // per-axis upper-face ordinals of the tile lattice
  int nface[3] = {0, 0, 0};
  double* d_tab = nullptr;
  int* d_fo = nullptr;
  const void* fwd_ws = nullptr;   // workspace holding the last forward's data
  std::string err;
  // sampled kernel timing
  int tstride = 0;
  long long launches[FWI_K_NCLASS] = {};
  std::vector<std::pair<hipEvent_t, hipEvent_t>> ev[FWI_K_NCLASS];
  size_t ev_used[FWI_K_NCLASS] = {};
  // second stream for the interior bricks, which run beside the PML bricks
  // (fork and join through events on the caller's stream)
  hipStream_t side = nullptr;
  hipEvent_t fork_ev = nullptr, join_ev = nullptr;
  // third stream: the second PML part beside the first (PMLFWI_CONCURRENT 2)
  hipStream_t side2 = nullptr;
  hipEvent_t join2_ev = nullptr;
  // largest eigenvalues of M^{-1} K for the unit reference brick with lam = 1,
  // mu = 0 and lam = 0, mu = 1 (stability bound of fwi_check_model)
  double c_lam = 0.0, c_mu = 0.0;
  double* d_info = nullptr;   // 8 doubles: model check [0, 5), power iteration [5, 8)
  double* d_partials = nullptr;   // MISFIT_BLOCKS doubles: per-workgroup misfit sums
  double* h_info = nullptr;       // 8 doubles of pinned host memory: copy of d_info
  int device = 0;                 // device current at fwi_plan_create
  Schedule sched;                 // checkpoint schedule (ckpt_every > 0)
  void* scratch = nullptr;        // device address of the fixed scratch array on that device
};

namespace {
// Brackets one kernel launch with events when it is a sampled launch.
struct TimedLaunch {
  fwi_plan* p;
  int cls;
  hipStream_t st;
  hipEvent_t stop = nullptr;
  TimedLaunch(fwi_plan* p_, int c, hipStream_t s) : p(p_), cls(c), st(s) {
    if (p->tstride <= 0) return;
    const long long n = p->launches[cls]++;
    if (n % p->tstride) return;
    auto& v = p->ev[cls];
    if (p->ev_used[cls] == v.size()) {
      std::pair<hipEvent_t, hipEvent_t> e{};
      if (hipEventCreate(&e.first) != hipSuccess || hipEventCreate(&e.second) != hipSuccess) return;
      v.push_back(e);
    }
    auto& e = v[p->ev_used[cls]++];
    (void)hipEventRecord(e.first, st);
    stop = e.second;
  }
  ~TimedLaunch() {
    if (stop) (void)hipEventRecord(stop, st);
  }
};
}  // namespace

namespace {

// Element tiles (bricks per axis; 5x4x2 measured fastest on the 5-brick PML
// and 40x40x20-brick interior workload among 4x2x2 .. 10x1x1 at 256-640
// threads) and whether a workgroup walks all sources of its tile (true) or one
// source per workgroup (false).
#ifndef PMLFWI_TX
#define PMLFWI_TX 5
#define PMLFWI_TY 4
#define PMLFWI_TZ 2
#endif
// PML operator as two launches, one per row type (smaller LDS and register
// footprints, 8 waves per SIMD; they interleave with the interior launch on
// the other stream), rather than one launch for both.  Forward stages launch
// the S-rows first, transposed stages the u-rows first: in each order the PML
// pair and the interior launch beside it end closest together.
#ifndef PMLFWI_PML_SPLIT
#define PMLFWI_PML_SPLIT 1
#endif
// Nodal launch: 0 one grid, 1 one grid with the (heavier) PML-row blocks
// dispatched first, 2 node rows and PML rows as two launches.
#ifndef PMLFWI_NODAL_ORDER
#define PMLFWI_NODAL_ORDER 1
#endif
#ifndef PMLFWI_SPLIT_FIRST_FWD
#define PMLFWI_SPLIT_FIRST_FWD PML_SROWS
#endif
#ifndef PMLFWI_SPLIT_FIRST_ADJ
#define PMLFWI_SPLIT_FIRST_ADJ PML_UROWS
#endif
#ifndef PMLFWI_CONCURRENT
#define PMLFWI_CONCURRENT 1
#endif
#ifndef PMLFWI_SRCLOOP
#define PMLFWI_SRCLOOP false
#endif
constexpr int TX = PMLFWI_TX, TY = PMLFWI_TY, TZ = PMLFWI_TZ;
constexpr bool SRCLOOP = PMLFWI_SRCLOOP;
constexpr int ETHREADS = PMLFWI_ETHREADS;   // threads per element workgroup

fwi_status fail(fwi_plan* p, fwi_status s, const std::string& msg) {
  if (p) p->err = msg;
  return s;
}

#define HIP_TRY(plan, call)                                                   \
  do {                                                                        \
    hipError_t e_ = (call);                                                   \
    if (e_ != hipSuccess)                                                     \
      return fail(plan, FWI_ERR_HIP, std::string(#call ": ") + hipGetErrorString(e_)); \
  } while (0)

Geo make_geo(const fwi_problem& P) {
  Geo g{};
  g.ex = P.ne_int[0]; g.ey = P.ne_int[1]; g.ez = P.ne_int[2];
  g.ps = P.npml_side; g.pb = P.npml_bottom;
  g.EX = g.ex + 2 * g.ps; g.EY = g.ey + 2 * g.ps; g.EZ = g.ez + g.pb;
  g.NX = 2 * g.EX + 1; g.NY = 2 * g.EY + 1; g.NZ = 2 * g.EZ + 1;
  g.NIX = 2 * g.ex + 1; g.NIY = 2 * g.ey + 1; g.NIZ = 2 * g.ez + 1;
  g.w = 2 * g.ps + 1; g.zb = 2 * g.pb;
  g.plane = g.NX * g.NY;
  g.ring = 2 * g.w * g.NX + (g.NY - 2 * g.w) * 2 * g.w;
  g.n_nodes = g.plane * g.NZ;
  g.n_pml = (g.zb + 1) * g.plane + (g.NZ - g.zb - 1) * g.ring;
  g.n_int = g.NIX * g.NIY * g.NIZ;
  g.sn = (g.n_nodes + 63) & ~63;
  g.sp = (g.n_pml + 63) & ~63;
  g.si = (g.n_int + 63) & ~63;
  g.h = P.h;
  g.hx = 0.5 * g.ex * P.h; g.hy = 0.5 * g.ey * P.h; g.hz = g.ez * P.h;
  g.Lps = g.ps * P.h; g.Lpb = g.pb * P.h;
  g.x0 = -(g.hx + g.Lps); g.y0 = -(g.hy + g.Lps); g.z0 = -(g.hz + g.Lpb);
  g.alpha0 = P.pml_alpha0; g.beta0 = P.pml_beta0; g.m = P.pml_m;
  return g;
}

// Per-axis brick segments: the interior range cut into chunks of T from its
// lower end, each PML range cut into chunks of T away from the interior.
struct Seg { int start, count; bool interior; };

std::vector<Seg> axis_segments(int lo_pml, int n_int, int hi_pml, int T) {
  std::vector<Seg> s;
  for (int e = lo_pml; e > 0; e -= T) s.push_back({std::max(0, e - T), e - std::max(0, e - T), false});
  for (int e = lo_pml; e < lo_pml + n_int; e += T)
    s.push_back({e, std::min(T, lo_pml + n_int - e), true});
  for (int e = lo_pml + n_int; e < lo_pml + n_int + hi_pml; e += T)
    s.push_back({e, std::min(T, lo_pml + n_int + hi_pml - e), false});
  return s;
}

// Largest eigenvalue of M^{-1} K for the reference brick [-1,1]^3 with the
// 3x3x3 LGL rule, K = sum_q w_q (lam (div)^T div + mu 2 eps^T : eps), M the
// lumped mass diag(w_a) per component; symmetric power iteration on
// M^{-1/2} K M^{-1/2} (host, 81 x 81).
double reference_eigen(double lam, double mu) {
  const double w1[3] = {1.0 / 3, 4.0 / 3, 1.0 / 3};
  const double D[3][3] = {{-1.5, 2.0, -0.5}, {-0.5, 0.0, 0.5}, {0.5, -2.0, 1.5}};   // D[q][a]
  std::vector<double> K(81 * 81, 0.0);
  for (int q = 0; q < 27; ++q) {
    const int qi[3] = {q % 3, (q / 3) % 3, q / 9};
    const double wq = w1[qi[0]] * w1[qi[1]] * w1[qi[2]];
    // G[k][i][col]: d_k u_i at q per unknown col = 3 a + i
    std::vector<double> G(9 * 81, 0.0);
    for (int k = 0; k < 3; ++k)
      for (int a = 0; a < 3; ++a) {
        int ai[3] = {qi[0], qi[1], qi[2]};
        ai[k] = a;
        const int node = ai[0] + 3 * ai[1] + 9 * ai[2];
        for (int i = 0; i < 3; ++i) G[(3 * k + i) * 81 + 3 * node + i] += D[qi[k]][a];
      }
    for (int r = 0; r < 81; ++r)
      for (int c = 0; c < 81; ++c) {
        const double divr = G[0 * 81 + r] + G[4 * 81 + r] + G[8 * 81 + r];
        const double divc = G[0 * 81 + c] + G[4 * 81 + c] + G[8 * 81 + c];
        double ee = 0.0;
        for (int i = 0; i < 3; ++i)
          for (int k = 0; k < 3; ++k) {
            const double er = 0.5 * (G[(3 * k + i) * 81 + r] + G[(3 * i + k) * 81 + r]);
            const double ec = 0.5 * (G[(3 * k + i) * 81 + c] + G[(3 * i + k) * 81 + c]);
            ee += er * ec;
          }
        K[r * 81 + c] += wq * (lam * divr * divc + mu * 2.0 * ee);
      }
  }
  std::vector<double> isq(81);
  for (int a = 0; a < 27; ++a)
    for (int i = 0; i < 3; ++i) isq[3 * a + i] = 1.0 / std::sqrt(w1[a % 3] * w1[(a / 3) % 3] * w1[a / 9]);
  std::vector<double> x(81), y(81);
  for (int r = 0; r < 81; ++r) x[r] = 1.0 + 0.01 * r;
  double ev = 0.0;
  for (int it = 0; it < 3000; ++it) {
    double nrm = 0.0;
    for (int r = 0; r < 81; ++r) {
      double acc = 0.0;
      for (int c = 0; c < 81; ++c) acc += K[r * 81 + c] * isq[c] * x[c];
      y[r] = isq[r] * acc;
      nrm += y[r] * y[r];
    }
    nrm = std::sqrt(nrm);
    double dot = 0.0;
    for (int r = 0; r < 81; ++r) dot += x[r] * y[r];
    double xx = 0.0;
    for (int r = 0; r < 81; ++r) xx += x[r] * x[r];
    ev = dot / xx;
    for (int r = 0; r < 81; ++r) x[r] = y[r] / nrm;
  }
  return ev;
}

void build_tiles(fwi_plan* p) {
  const Geo& g = p->g;
  auto sx = axis_segments(g.ps, g.ex, g.ps, TX);
  auto sy = axis_segments(g.ps, g.ey, g.ps, TY);
  auto sz = axis_segments(g.pb, g.ez, 0, TZ);
  for (auto& c : sz)
    for (auto& b : sy)
      for (auto& a : sx) {
        Tile t{a.start, b.start, c.start, a.count | (b.count << 8) | (c.count << 16)};
        if (a.interior && b.interior && c.interior) p->tiles_int.push_back(t);
        else p->tiles_pml.push_back(t);
      }
  // upper faces of the lattice, numbered in increasing order per axis
  const int nt = g.NX + g.NY + g.NZ;
  p->fo.assign(nt, -1);
  const std::vector<Seg>* segs[3] = {&sx, &sy, &sz};
  const int off[3] = {0, g.NX, g.NX + g.NY};
  for (int d = 0; d < 3; ++d) {
    std::vector<int> faces;
    for (auto& a : *segs[d]) faces.push_back(2 * (a.start + a.count));
    std::sort(faces.begin(), faces.end());
    for (size_t f = 0; f < faces.size(); ++f) p->fo[off[d] + faces[f]] = (int)f;
    p->nface[d] = (int)faces.size();
  }
  // per-axis PML profile and lumped-mass factors (double, host)
  p->tab.assign(4 * (size_t)nt, 0.0);
  for (int l = 0; l < g.NX; ++l) {
    stretch(g, fabs(g.x0 + 0.5 * g.h * l) - g.hx, g.Lps, p->tab[l], p->tab[nt + l]);
    p->tab[2 * nt + l] = mass1d(l, 0, g.EX);
    p->tab[3 * nt + l] = mass1d(l, g.ps, g.ps + g.ex);
  }
  for (int l = 0; l < g.NY; ++l) {
    const int o = g.NX + l;
    stretch(g, fabs(g.y0 + 0.5 * g.h * l) - g.hy, g.Lps, p->tab[o], p->tab[nt + o]);
    p->tab[2 * nt + o] = mass1d(l, 0, g.EY);
    p->tab[3 * nt + o] = mass1d(l, g.ps, g.ps + g.ey);
  }
  for (int l = 0; l < g.NZ; ++l) {
    const int o = g.NX + g.NY + l;
    stretch(g, -(g.z0 + 0.5 * g.h * l) - g.hz, g.Lpb, p->tab[o], p->tab[nt + o]);
    p->tab[2 * nt + o] = mass1d(l, 0, g.EZ);
    p->tab[3 * nt + o] = mass1d(l, g.pb, g.EZ);
  }
}

// Partial-array layouts: residual (9 rows per node) and gradient (2 per node).
Part part_layout(const Geo& g, const int nface[3], int rows, bool pml_compact0) {
  Part P{};
  long long o = 0;
  for (int c = 0; c < 8; ++c) {
    const int nx = (c & 1) ? nface[0] : g.NX;
    const int ny = (c & 2) ? nface[1] : g.NY;
    const int nz = (c & 4) ? nface[2] : g.NZ;
    P.nx[c] = nx;
    P.ny[c] = ny;
    // c != 0 strides rounded up to 64 entries (256-byte aligned rows); array 0
    // of the residual uses the register index spaces
    P.size[c] = c == 0 ? (long long)g.sn : (((long long)nx * ny * nz + 63) & ~63LL);
    P.off[c] = o;
    o += (c == 0 && pml_compact0) ? 3LL * g.sn + 6LL * g.sp : (long long)rows * P.size[c];
  }
  P.per_src = o;
  return P;
}

// ---------------------------------------------------------------- sizes
struct Layout {
  size_t es;          // element size of the state type
  size_t reg_elems;   // one register, one source
  size_t res_elems;   // residual, one source
  size_t stage_elems; // stored stage displacement, all sources
  size_t pstage_elems;// stored stage PML displacement fields, all sources (full gradient)
  int nreg, nstore, nckpt;
  size_t off_lam, off_mu, off_invm, off_regs, off_res, off_gacc, off_store, off_pstore, off_ckpt, total;
  Part part, gpart;
};

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

int count_faces(const fwi_problem& P, const Geo& g, int d) {
  if (d == 0) return (int)axis_segments(g.ps, g.ex, g.ps, TX).size();
  if (d == 1) return (int)axis_segments(g.ps, g.ey, g.ps, TY).size();
  return (int)axis_segments(g.pb, g.ez, 0, TZ).size();
}

// keep = false: a forward solve that keeps nothing for the adjoint (no stage
// store, no checkpoints, no gradient accumulators).
Layout layout(const fwi_problem& P, const Geo& g, bool keep = true) {
  Layout L{};
  keep = keep && P.ckpt_every >= 0;   // ckpt_every < 0: forward-only plan
  const int nface[3] = {count_faces(P, g, 0), count_faces(P, g, 1), count_faces(P, g, 2)};
  L.part = part_layout(g, nface, 9, true);
  L.gpart = part_layout(g, nface, 2, false);
  L.es = P.precision == FWI_FP64 ? 8 : 4;
  L.reg_elems = (size_t)U_NCOMP * g.sn + (size_t)P_NCOMP * g.sp;
  L.res_elems = 3 * (size_t)g.sn + 6 * (size_t)g.sp;
  L.stage_elems = (size_t)P.nsrc * 3 * g.si;
  L.pstage_elems = P.grad_full ? (size_t)P.nsrc * 9 * g.sp : 0;
  const int k = P.ckpt_every;
  L.nreg = (k == 0 || !keep) ? 4 : 8;
  L.nstore = !keep ? 0 : (k == 0 ? P.nsteps : std::min(k, P.nsteps));
  if (k > 0 && keep) {
    const int nseg = (P.nsteps + k - 1) / k;
    L.nckpt = (P.ckpt_slots == 0 || P.ckpt_slots >= nseg - 1) ? nseg : P.ckpt_slots;
  } else {
    L.nckpt = 0;
  }
  size_t o = 0;
  L.off_lam = o; o = align256(o + (size_t)g.n_int * L.es);
  L.off_mu = o; o = align256(o + (size_t)g.n_int * L.es);
  L.off_invm = o; o = align256(o + (size_t)g.n_nodes * L.es);
  L.off_regs = o; o = align256(o + (size_t)L.nreg * P.nsrc * L.reg_elems * L.es);
  L.off_res = o; o = align256(o + (size_t)P.nsrc * L.part.per_src * L.es);
  L.off_gacc = o; o = align256(o + (keep ? (size_t)L.gpart.per_src * sizeof(double) : 0));
  L.off_store = o; o = align256(o + (size_t)L.nstore * 4 * L.stage_elems * L.es);
  L.off_pstore = o; o = align256(o + (size_t)L.nstore * 4 * L.pstage_elems * L.es);
  L.off_ckpt = o; o = align256(o + (size_t)L.nckpt * P.nsrc * L.reg_elems * L.es);
  L.total = o;
  return L;
}

fwi_status validate(const fwi_problem* P) {
  if (!P) return FWI_ERR_ARG;
  for (int d = 0; d < 3; ++d)
    if (P->ne_int[d] < 1) return FWI_ERR_SHAPE;
  if (P->npml_side < 1 || P->npml_bottom < 1) return FWI_ERR_SHAPE;
  if (!(P->h > 0) || !(P->dt > 0) || P->nsteps < 1) return FWI_ERR_ARG;
  if (P->nsrc < 1 || P->nrec < 0 || P->pml_m < 0 || P->ckpt_every < -1) return FWI_ERR_ARG;
  if (P->precision < FWI_FP64 || P->precision > FWI_FP32_BF16X3) return FWI_ERR_ARG;
  if (P->grad_full != 0 && P->grad_full != 1) return FWI_ERR_ARG;
  if (P->ckpt_slots < 0 || (P->ckpt_slots > 0 && P->ckpt_every <= 0)) return FWI_ERR_ARG;
  const double nx = 2.0 * (P->ne_int[0] + 2.0 * P->npml_side) + 1;
  const double ny = 2.0 * (P->ne_int[1] + 2.0 * P->npml_side) + 1;
  const double nz = 2.0 * (P->ne_int[2] + P->npml_bottom) + 1;
  if (nx * ny * nz * 21.0 > 2147483647.0) return FWI_ERR_SHAPE;   // 32-bit node indexing
  return FWI_OK;
}

// ---------------------------------------------------------------- small kernels
template <typename T>
__global__ void fill_kernel(T* p, size_t n, T v) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    p[i] = v;
}

template <typename R>
__global__ void convert_kernel(const double* __restrict__ in, R* __restrict__ out, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = R(in[i]);
}

template <typename R>
__global__ void receivers_kernel(const R* __restrict__ X, long long reg, int sn,
                                 const int* __restrict__ rec, int nrec, double* __restrict__ traces,
                                 int step, int nsteps) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x, src = blockIdx.y;
  if (r >= nrec) return;
  const R* U = X + (size_t)src * reg;
  double* T = traces + ((size_t)src * (nsteps + 1) + step) * nrec * 3 + (size_t)r * 3;
  const int node = rec[r];
  for (int d = 0; d < 3; ++d) T[d] = (double)U[u_at(sn, d, node)];
}

// Adjoint impulse after a reverse step: y2_u += M^{-1} dt w_n (u^n - u_m^n) at receivers.
template <typename R>
__global__ void impulse_kernel(R* __restrict__ Y, long long reg, int sn, const R* __restrict__ invMu,
                               const int* __restrict__ rec, int nrec, const double* __restrict__ resid,
                               int step, int nsteps, double scale) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x, src = blockIdx.y;
  if (r >= nrec) return;
  R* U = Y + (size_t)src * reg;
  const double* E = resid + ((size_t)src * (nsteps + 1) + step) * nrec * 3 + (size_t)r * 3;
  const int node = rec[r];
  const R im = invMu[node];
  for (int d = 0; d < 3; ++d) atomic_add(&U[u_at(sn, 3 + d, node)], R(scale * E[d]) * im);
}

// Receiver forcing of the paper's reverse RK4 (App. B) in one stage.  With
// z = (y0, -y1, y2) the scheme is classical RK4 on the transposed operator
// plus the rate -M^{-1} R^T r(t) in the x2 rows, r(t) = a_hi r_hi + a_lo r_lo
// at the stage time; the stage combination the nodal kernel just applied gets
// that rate's share: mode 0/1: Yout += cY g, acc += cA g; mode 2: Xn += cA g.
template <typename R>
__global__ void appb_force_kernel(R* __restrict__ Yout, R* __restrict__ Xn, R* __restrict__ acc, long long reg,
                                  int sn, int mode, double cA, double cY, const R* __restrict__ invMu,
                                  const int* __restrict__ rec, int nrec, const double* __restrict__ resid,
                                  int n_hi, int n_lo, double a_hi, double a_lo, int nsteps) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x, src = blockIdx.y;
  if (r >= nrec) return;
  const size_t off = (size_t)src * reg;
  const double* Eh = resid + ((size_t)src * (nsteps + 1) + n_hi) * nrec * 3 + (size_t)r * 3;
  const double* El = resid + ((size_t)src * (nsteps + 1) + n_lo) * nrec * 3 + (size_t)r * 3;
  const int node = rec[r];
  const double im = (double)invMu[node];
  for (int d = 0; d < 3; ++d) {
    const double gval = -im * (a_hi * Eh[d] + a_lo * El[d]);
    const size_t o = off + u_at(sn, 3 + d, node);
    if (mode == 2) {
      atomic_add(&Xn[o], R(cA * gval));
    } else {
      atomic_add(&Yout[o], R(cY * gval));
      atomic_add(&acc[o], R(cA * gval));
    }
  }
}

// Misfit (7): residual and per-workgroup sums of w_n r^2 (trapezoid weights),
// then one workgroup adds the partial sums in a fixed order, so J has the same
// bits on every run (the grid size depends only on the trace length).
constexpr int MISFIT_BLOCKS = 2048;

// General nodal loads after a nodal stage pass: the stage rate of x2 at the
// load's node gains M^{-1} f, f = vec * wavelet(stage time); the stage
// combination the nodal kernel applied gets that rate's share (mode 0/1:
// Yout += cY g, acc += cA g; mode 2: Xn += cA g).  Entries are unique per
// (source, node), so plain read-modify-writes do not race.
template <typename R>
__global__ void load_kernel(R* __restrict__ Yout, R* __restrict__ Xn, R* __restrict__ acc, long long reg, int sn,
                            int mode, double cA, double cY, const R* __restrict__ invMu, int nload,
                            const int* __restrict__ lsrc, const int* __restrict__ lnode,
                            const double* __restrict__ lvec, const double* __restrict__ wav, int wav_len,
                            int wav_idx) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= nload) return;
  const int src = lsrc[e], node = lnode[e];
  const double f = wav[(size_t)src * wav_len + wav_idx];
  const double im = (double)invMu[node];
  const size_t off = (size_t)src * reg;
  for (int d = 0; d < 3; ++d) {
    const double g = im * lvec[3 * e + d] * f;
    const size_t o = off + u_at(sn, 3 + d, node);
    if (mode == 2) {
      Xn[o] += R(cA * g);
    } else {
      Yout[o] += R(cY * g);
      acc[o] += R(cA * g);
    }
  }
}

__global__ void __launch_bounds__(256) misfit_kernel(const double* __restrict__ tr, const double* __restrict__ obs,
                                                     double* __restrict__ resid, long long n, int per_step,
                                                     int nsteps, double* __restrict__ partials) {
  __shared__ double part[256];
  double acc = 0.0;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
    const double r = tr[i] - obs[i];
    resid[i] = r;
    const int step = (int)((i / per_step) % (nsteps + 1));
    const double w = (step == 0 || step == nsteps) ? 0.5 : 1.0;
    acc += w * r * r;
  }
  part[threadIdx.x] = acc;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) part[threadIdx.x] += part[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) partials[blockIdx.x] = part[0];
}

__global__ void __launch_bounds__(256) misfit_final_kernel(const double* __restrict__ partials, int nb,
                                                           double half_dt, double* __restrict__ J) {
  __shared__ double part[256];
  double acc = 0.0;
  for (int b = threadIdx.x; b < nb; b += blockDim.x) acc += partials[b];
  part[threadIdx.x] = acc;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) part[threadIdx.x] += part[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) J[0] = half_dt * part[0];
}

// x1 displacement of a register on the interior closure -> stage store slot.
template <typename R>
__global__ void extract_kernel(Geo g, const R* __restrict__ X, long long reg, R* __restrict__ S, long long sstr) {
  const int mi = blockIdx.x * blockDim.x + threadIdx.x, src = blockIdx.y;
  if (mi >= g.n_int) return;
  const int jz = mi / (g.NIX * g.NIY), rr = mi - jz * g.NIX * g.NIY, jy = rr / g.NIX, jx = rr - jy * g.NIX;
  const size_t node = (size_t)(jx + 2 * g.ps) + (size_t)g.NX * ((jy + 2 * g.ps) + (size_t)g.NY * (jz + 2 * g.pb));
  for (int d = 0; d < 3; ++d)
    S[(size_t)src * sstr + 3 * (size_t)mi + d] = X[(size_t)src * reg + u_at(g.sn, d, node)];
}

// PML displacement fields of a register -> stored-stage slot [x1 u | x2 u | x0 u] x sp
// (zero on Dirichlet nodes; x0 u only on history nodes).
template <typename R>
__global__ void pextract_kernel(Geo g, const R* __restrict__ X, long long reg, R* __restrict__ S, long long sstr) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x, src = blockIdx.y;
  if (p >= g.n_pml) return;
  int i, j, k;
  pml_coords(g, p, i, j, k);
  const size_t node = (size_t)i + (size_t)g.NX * (j + (size_t)g.NY * k);
  const R* U = X + (size_t)src * reg;
  const R* P = U + 6 * (size_t)g.sn;
  R* D = S + (size_t)src * sstr;
  const bool dir = is_dirichlet(g, i, j, k);
  const bool hist = !dir && pml_coef_tab(g, i, j, k).nbeta >= 2;
  for (int d = 0; d < 3; ++d) {
    D[(size_t)d * g.sp + p] = dir ? R(0) : U[u_at(g.sn, d, node)];
    D[(size_t)(3 + d) * g.sp + p] = dir ? R(0) : U[u_at(g.sn, 3 + d, node)];
    D[(size_t)(6 + d) * g.sp + p] = hist ? P[p_at(g.sp, P_X0U + d, p)] : R(0);
  }
}

// g = sum over the PML and interior nodes that take their material from
// interior node mi (the node itself and, on the interface, the PML nodes that
// project onto it) of the accumulator slots that can hold a contribution.
__global__ void gradient_reduce_full_kernel(Geo g, const double* __restrict__ gacc, Part PG,
                                            double* __restrict__ g_lam, double* __restrict__ g_mu) {
  const int mi = blockIdx.x * blockDim.x + threadIdx.x;
  if (mi >= g.n_int) return;
  const int jz = mi / (g.NIX * g.NIY), rr = mi - jz * g.NIX * g.NIY, jy = rr / g.NIX, jx = rr - jy * g.NIX;
  auto range = [](int jm, int n_int, int off, int n_full, int& lo, int& hi) {
    lo = jm + off;
    hi = jm + off;
    if (jm == 0) lo = 0;
    if (jm == n_int - 1) hi = n_full - 1;
  };
  int i0, i1, j0, j1, k0, k1;
  range(jx, g.NIX, 2 * g.ps, g.NX, i0, i1);
  range(jy, g.NIY, 2 * g.ps, g.NY, j0, j1);
  range(jz, g.NIZ, 2 * g.pb, g.NZ, k0, k1);
  double a = 0.0, b = 0.0;
  for (int k = k0; k <= k1; ++k)
    for (int j = j0; j <= j1; ++j)
      for (int i = i0; i <= i1; ++i) {
        const int mask = face_mask(g, i, j, k);
        size_t o = (size_t)PG.off[0] + part_node(g, PG, 0, i, j, k);
        a += gacc[o];
        b += gacc[o + PG.size[0]];
        for (int c = mask; c; c = (c - 1) & mask) {
          o = (size_t)PG.off[c] + part_node(g, PG, c, i, j, k);
          a += gacc[o];
          b += gacc[o + PG.size[c]];
        }
      }
  g_lam[mi] = a;
  g_mu[mi] = b;
}

// g = sum of the gradient accumulator slots that can hold a contribution.
__global__ void gradient_reduce_kernel(Geo g, const double* __restrict__ gacc, Part PG,
                                       double* __restrict__ g_lam, double* __restrict__ g_mu) {
  const int mi = blockIdx.x * blockDim.x + threadIdx.x;
  if (mi >= g.n_int) return;
  const int jz = mi / (g.NIX * g.NIY), rr = mi - jz * g.NIX * g.NIY, jy = rr / g.NIX, jx = rr - jy * g.NIX;
  const int i = jx + 2 * g.ps, j = jy + 2 * g.ps, k = jz + 2 * g.pb;
  const int mask = face_mask(g, i, j, k);
  size_t o = (size_t)PG.off[0] + part_node(g, PG, 0, i, j, k);
  double a = gacc[o], b = gacc[o + PG.size[0]];
  for (int c = mask; c; c = (c - 1) & mask) {
    o = (size_t)PG.off[c] + part_node(g, PG, c, i, j, k);
    a += gacc[o];
    b += gacc[o + PG.size[c]];
  }
  g_lam[mi] = a;
  g_mu[mi] = b;
}

// out = [min rho, min mu, min (3 lam + 2 mu), max vp, max over interior bricks of
// (max(lam, 0) c_lam + max mu c_mu) / min rho] (nodal values of each brick):
// one workgroup, fixed order.
__global__ void __launch_bounds__(1024) model_check_kernel(Geo g, const double* __restrict__ rho,
                                                           const double* __restrict__ lam,
                                                           const double* __restrict__ mu, double c_lam,
                                                           double c_mu, double* __restrict__ out) {
  __shared__ double red[5][1024];
  double mr = 1e300, mm = 1e300, mk = 1e300, vp = 0.0, wb = 0.0;
  for (int j = threadIdx.x; j < g.n_int; j += blockDim.x) {
    mr = fmin(mr, rho[j]);
    mm = fmin(mm, mu[j]);
    mk = fmin(mk, 3.0 * lam[j] + 2.0 * mu[j]);
    if (rho[j] > 0.0 && lam[j] + 2.0 * mu[j] > 0.0) vp = fmax(vp, sqrt((lam[j] + 2.0 * mu[j]) / rho[j]));
  }
  const long long nb = (long long)g.ex * g.ey * g.ez;
  for (long long e = threadIdx.x; e < nb; e += blockDim.x) {
    const int ex = (int)(e % g.ex), ey = (int)((e / g.ex) % g.ey), ez = (int)(e / ((long long)g.ex * g.ey));
    double lmax = 0.0, mmax = 0.0, rmin = 1e300;
    for (int c = 0; c < 27; ++c) {
      const int j = (2 * ex + c % 3) + g.NIX * ((2 * ey + (c / 3) % 3) + g.NIY * (2 * ez + c / 9));
      lmax = fmax(lmax, lam[j]);
      mmax = fmax(mmax, mu[j]);
      rmin = fmin(rmin, rho[j]);
    }
    if (rmin > 0.0) wb = fmax(wb, (lmax * c_lam + mmax * c_mu) / rmin);
  }
  red[0][threadIdx.x] = mr;
  red[1][threadIdx.x] = mm;
  red[2][threadIdx.x] = mk;
  red[3][threadIdx.x] = vp;
  red[4][threadIdx.x] = wb;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) {
      for (int k = 0; k < 3; ++k) red[k][threadIdx.x] = fmin(red[k][threadIdx.x], red[k][threadIdx.x + s]);
      for (int k = 3; k < 5; ++k) red[k][threadIdx.x] = fmax(red[k][threadIdx.x], red[k][threadIdx.x + s]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0)
    for (int k = 0; k < 5; ++k) out[k] = red[k][0];
}

// Power iteration for the largest eigenvalue of M_RD^{-1} K_RD, the interior
// stiffness over the lumped interior mass (the operator the RK4 stability
// limit is set by; the PML stretching only adds mass).  Iterate x (x1
// displacement of a register, source 0) was produced unscaled; with s the
// scale stored by the previous reduction, x s has unit M_RD norm.  r = K x is
// in the partial arrays (interior bricks only).  Per workgroup: sums of
// x.r, m x.x and m y.y with y = r / m; writes y s to the next register.
__device__ __forceinline__ double power_start(unsigned node, int d) {
  // deterministic start vector in [-1, 1): integer hash of (node, component)
  unsigned long long z = (unsigned long long)node * 3ULL + (unsigned long long)d + 0x9E3779B97F4A7C15ULL;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  z ^= z >> 31;
  return (double)(z >> 11) * (2.0 / 9007199254740992.0) - 1.0;
}

template <typename R>
__global__ void __launch_bounds__(256) power_step_kernel(Geo g, const R* __restrict__ X, R* __restrict__ Y,
                                                         const R* __restrict__ res, Part PT,
                                                         const double* __restrict__ rho, int first,
                                                         const double* __restrict__ state,
                                                         double* __restrict__ partials) {
  __shared__ double red[3][256];
  const double sc = first ? 1.0 : state[0];
  double xr = 0.0, xm = 0.0, ym = 0.0;
  for (int node = blockIdx.x * blockDim.x + threadIdx.x; node < g.n_nodes; node += gridDim.x * blockDim.x) {
    const int k = node / g.plane, r_ = node - k * g.plane, j = r_ / g.NX, i = r_ - j * g.NX;
    if (is_dirichlet(g, i, j, k)) continue;
    const int mi = interior_index(g, i, j, k);
    if (mi < 0) continue;
    double mrd, mp;
    lumped_masses_tab(g, i, j, k, mrd, mp);
    const double m = rho[mi] * mrd;
    const PartSlots PS = part_slots(g, PT, i, j, k);
    R r3[3];
    gather_rows<R, 3, false>(PT, PS, res, 3 * (size_t)node, r3);
    for (int d = 0; d < 3; ++d) {
      const size_t o = u_at(g.sn, d, node);
      const double x = (double)X[o] * sc;
      const double r = (double)r3[d] * sc;
      xr += x * r;
      xm += m * x * x;
      const double y = r / m;
      ym += m * y * y;
      Y[o] = R(y);
    }
  }
  red[0][threadIdx.x] = xr;
  red[1][threadIdx.x] = xm;
  red[2][threadIdx.x] = ym;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s)
      for (int c = 0; c < 3; ++c) red[c][threadIdx.x] += red[c][threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0)
    for (int c = 0; c < 3; ++c) partials[3 * blockIdx.x + c] = red[c][0];
}

// Fixed-order sum of the partials: state[0] = scale of the next iterate
// (1 / |y|_M), state[1] = Rayleigh quotient x.Kx / x.Mx, running maximum in state[2].
__global__ void __launch_bounds__(256) power_reduce_kernel(const double* __restrict__ partials, int nb,
                                                           double* __restrict__ state) {
  __shared__ double red[3][256];
  double a[3] = {0.0, 0.0, 0.0};
  for (int b = threadIdx.x; b < nb; b += blockDim.x)
    for (int c = 0; c < 3; ++c) a[c] += partials[3 * b + c];
  for (int c = 0; c < 3; ++c) red[c][threadIdx.x] = a[c];
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s)
      for (int c = 0; c < 3; ++c) red[c][threadIdx.x] += red[c][threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double rq = red[1][0] > 0.0 ? red[0][0] / red[1][0] : 0.0;
    state[0] = red[2][0] > 0.0 ? 1.0 / sqrt(red[2][0]) : 0.0;
    state[1] = rq;
    state[2] = fmax(state[2], rq);
  }
}

// Start vector of the power iteration: deterministic values on the free
// interior-closure nodes, zero elsewhere (x1 displacement of a register).
template <typename R>
__global__ void power_init_kernel(Geo g, R* __restrict__ X, double* __restrict__ state) {
  const int node = blockIdx.x * blockDim.x + threadIdx.x;
  if (node == 0) state[2] = 0.0;
  if (node >= g.n_nodes) return;
  const int k = node / g.plane, r_ = node - k * g.plane, j = r_ / g.NX, i = r_ - j * g.NX;
  const bool on = !is_dirichlet(g, i, j, k) && interior_index(g, i, j, k) >= 0;
  for (int d = 0; d < 3; ++d) X[u_at(g.sn, d, node)] = on ? R(power_start((unsigned)node, d)) : R(0);
}

// Nodal test fields [nsrc][9][n_nodes] <-> register slot (0: x0, 1: x1, 2: x2).
template <typename R>
__global__ void pack_kernel(Geo g, const double* __restrict__ in, R* __restrict__ X, long long reg, int slot) {
  const int node = blockIdx.x * blockDim.x + threadIdx.x, src = blockIdx.y;
  if (node >= g.n_nodes) return;
  const int k = node / g.plane, r_ = node - k * g.plane, j = r_ / g.NX, i = r_ - j * g.NX;
  const size_t nf = g.n_nodes, nn = g.sn, np = g.sp;
  const double* F = in + (size_t)src * 9 * nf;
  R* U = X + (size_t)src * reg;
  R* P = U + 6 * nn;
  const bool dir = is_dirichlet(g, i, j, k), pml = in_pml(g, i, j, k);
  const size_t p = pml ? (size_t)pml_index(g, i, j, k) : 0;
  for (int d = 0; d < 3; ++d) {
    const R v = dir ? R(0) : R(F[d * nf + node]);
    if (slot == 0) { if (pml) P[p_at(np, P_X0U + d, p)] = v; }
    else U[u_at(nn, slot == 1 ? d : 3 + d, node)] = v;
  }
  if (pml) {
    const int base = slot == 0 ? P_X0S : (slot == 1 ? P_X1S : P_X2S);
    for (int v = 0; v < 6; ++v) P[p_at(np, base + v, p)] = R(F[(3 + v) * nf + node]);
  }
}

// out = -M^{-1}(r + nodal PML terms) for the register Y, nodal layout.
template <typename R>
__global__ void accel_kernel(Geo g, const R* __restrict__ Y, long long reg, const R* __restrict__ res,
                             Part PT, const R* __restrict__ invMu, double* __restrict__ out) {
  const int node = blockIdx.x * blockDim.x + threadIdx.x, src = blockIdx.y;
  if (node >= g.n_nodes) return;
  const int k = node / g.plane, r_ = node - k * g.plane, j = r_ / g.NX, i = r_ - j * g.NX;
  const size_t nf = g.n_nodes, nn = g.sn, np = g.sp;
  const R* U = Y + (size_t)src * reg;
  const R* P = U + 6 * nn;
  const R* rs = res + (size_t)src * PT.per_src;
  double* O = out + (size_t)src * 9 * nf;
  const bool dir = is_dirichlet(g, i, j, k), pml = in_pml(g, i, j, k);
  for (int c = 0; c < 9; ++c) O[c * nf + node] = 0.0;
  double mrd, mp;
  lumped_masses_tab(g, i, j, k, mrd, mp);
  const PmlCoef cf = pml_coef_tab(g, i, j, k);
  const size_t p = pml ? (size_t)pml_index(g, i, j, k) : 0;
  const bool hist = cf.nbeta >= 2;
  const PartSlots PS = part_slots(g, PT, i, j, k);
  if (!dir) {
    R r3[3];
    gather_rows<R, 3, false>(PT, PS, rs, 3 * (size_t)node, r3);
    for (int d = 0; d < 3; ++d) {
      double a = -(double)invMu[node] * (double)r3[d];
      if (pml) {
        const double kap = mp / (mrd + cf.a * mp);
        const double u0 = hist ? (double)P[p_at(np, P_X0U + d, p)] : 0.0;
        a -= kap * (cf.b * (double)U[u_at(nn, 3 + d, node)] + cf.c * (double)U[u_at(nn, d, node)] + cf.d * u0);
      }
      O[d * nf + node] = a;
    }
  }
  if (pml) {
    R r6[6];
    gather_rows<R, 6, true>(PT, PS, rs, 3 * nn + 6 * p, r6);
    for (int v = 0; v < 6; ++v) {
      const double s0 = hist ? (double)P[p_at(np, P_X0S + v, p)] : 0.0;
      O[(3 + v) * nf + node] = -(double)r6[v] / (cf.a * mp) -
                               (cf.b * (double)P[p_at(np, P_X2S + v, p)] + cf.c * (double)P[p_at(np, P_X1S + v, p)] +
                                cf.d * s0) / cf.a;
    }
  }
}

inline unsigned blocks(size_t n, int t) { return (unsigned)((n + t - 1) / t); }

// ---------------------------------------------------------------- step loops
template <typename R>
struct Run {
  fwi_plan* p;
  hipStream_t st;
  Layout L;
  char* ws;
  const Geo& g() const { return p->g; }
  R* lam() const { return (R*)(ws + L.off_lam); }
  R* mu() const { return (R*)(ws + L.off_mu); }
  R* invm() const { return (R*)(ws + L.off_invm); }
  R* reg(int r) const { return (R*)(ws + L.off_regs) + (size_t)r * p->nsrc * L.reg_elems; }
  R* res() const { return (R*)(ws + L.off_res); }
  double* gacc() const { return (double*)(ws + L.off_gacc); }
  R* pstore(int nl, int s) const {
    return L.pstage_elems ? (R*)(ws + L.off_pstore) + ((size_t)nl * 4 + s) * L.pstage_elems : nullptr;
  }
  R* store(int nl, int s) const {
    return (R*)(ws + L.off_store) + ((size_t)nl * 4 + s) * L.stage_elems;
  }
  R* ckpt(int c) const { return (R*)(ws + L.off_ckpt) + (size_t)c * p->nsrc * L.reg_elems; }

  template <typename T>
  fwi_status fill(T* ptr, size_t n, T v) {
    if (n == 0) return FWI_OK;
    const unsigned nb = std::min<size_t>(blocks(n, 256), 65536);
    fill_kernel<T><<<nb, 256, 0, st>>>(ptr, n, v);
    HIP_TRY(p, hipGetLastError());
    return FWI_OK;
  }

  fwi_status setup(const double* rho, const double* lam, const double* mu) {
    const Geo& G = g();
    convert_kernel<R><<<blocks(G.n_int, 256), 256, 0, st>>>(lam, this->lam(), G.n_int);
    convert_kernel<R><<<blocks(G.n_int, 256), 256, 0, st>>>(mu, this->mu(), G.n_int);
    inv_mass_kernel<R><<<blocks(G.n_nodes, 256), 256, 0, st>>>(G, rho, invm());
    HIP_TRY(p, hipGetLastError());
    return FWI_OK;
  }

  // Interior operator on the matrix cores for the FP32-state precisions that
  // ask for it; false when the scalar kernel is to be used.
  bool mfma_interior(const R* Y, int nt, unsigned gx, hipStream_t st) {
    if constexpr (std::is_same<R, float>::value) {
      const int pr = p->prob.precision;
      if (pr != FWI_FP32_MFMA && pr != FWI_FP32_BF16X3) return false;
      const dim3 grid(gx, p->nsrc);
      if (pr == FWI_FP32_MFMA)
        interior_mfma_kernel<MFMA_F32, TX, TY, TZ><<<grid, mfma_threads(MFMA_F32), 0, st>>>(
            g(), p->d_tiles_int, nt, Y, (long long)L.reg_elems, lam(), mu(), res(), L.part);
      else
        interior_mfma_kernel<MFMA_BF16X3, TX, TY, TZ><<<grid, mfma_threads(MFMA_BF16X3), 0, st>>>(
            g(), p->d_tiles_int, nt, Y, (long long)L.reg_elems, lam(), mu(), res(), L.part);
      return true;
    }
    return false;
  }

  // The interior and PML bricks write disjoint partial-array entries, so the
  // two launches may run at the same time: the interior one goes to the plan's
  // second stream when both lists are non-empty.
  // PML rows on the matrix cores for the FP32-state precisions that ask for it
  // (one source per workgroup, one row type per launch); false when the scalar
  // kernel is to be used.
  template <int PART>
  bool mfma_pml(bool adj, unsigned gx, int nt, const R* Y, long long reg, hipStream_t sp) {
    if constexpr (std::is_same<R, float>::value) {
      const int pr = p->prob.precision;
      if (pr != FWI_FP32_MFMA && pr != FWI_FP32_BF16X3) return false;
      if constexpr (PART == PML_ALL) {
        mfma_pml<PML_UROWS>(adj, gx, nt, Y, reg, sp);
        mfma_pml<PML_SROWS>(adj, gx, nt, Y, reg, sp);
      } else {
        const dim3 grid(gx, p->nsrc);
        const Tile* T = p->d_tiles_pml;
        if (pr == FWI_FP32_MFMA) {
          constexpr int th = mfma_threads(MFMA_F32);
          if (adj)
            pml_mfma_kernel<MFMA_F32, TX, TY, TZ, true, PART><<<grid, th, 0, sp>>>(g(), T, nt, Y, reg, lam(), mu(),
                                                                                 res(), L.part);
          else
            pml_mfma_kernel<MFMA_F32, TX, TY, TZ, false, PART><<<grid, th, 0, sp>>>(g(), T, nt, Y, reg, lam(), mu(),
                                                                                  res(), L.part);
        } else {
          constexpr int th = mfma_threads(MFMA_BF16X3);
          if (adj)
            pml_mfma_kernel<MFMA_BF16X3, TX, TY, TZ, true, PART><<<grid, th, 0, sp>>>(g(), T, nt, Y, reg, lam(),
                                                                                    mu(), res(), L.part);
          else
            pml_mfma_kernel<MFMA_BF16X3, TX, TY, TZ, false, PART><<<grid, th, 0, sp>>>(g(), T, nt, Y, reg, lam(),
                                                                                     mu(), res(), L.part);
        }
      }
      return true;
    }
    return false;
  }

  template <int PART>
  void launch_pml(bool adj, dim3 grid, int nt, const R* Y, long long reg, hipStream_t sp) {
    if (mfma_pml<PART>(adj, grid.x, nt, Y, reg, sp)) return;
    if (adj)
      pml_element_kernel<R, TX, TY, TZ, true, SRCLOOP, PART><<<grid, ETHREADS, 0, sp>>>(
          g(), p->d_tiles_pml, nt, p->nsrc, Y, reg, lam(), mu(), res(), L.part);
    else
      pml_element_kernel<R, TX, TY, TZ, false, SRCLOOP, PART><<<grid, ETHREADS, 0, sp>>>(
          g(), p->d_tiles_pml, nt, p->nsrc, Y, reg, lam(), mu(), res(), L.part);
  }

  fwi_status elements(bool adj, const R* Y, const R* fwd, double gw, bool interior_only = false,
                      const R* pfwd = nullptr) {
    const Geo& G = g();
    const long long reg = (long long)L.reg_elems;
    const int ns = p->nsrc;
    hipStream_t si = st;
    const bool pml = !interior_only && !p->tiles_pml.empty();
    const bool fork = PMLFWI_CONCURRENT && !p->tiles_int.empty() && pml;
    const bool fork2 = fork && PMLFWI_CONCURRENT == 2 && PMLFWI_PML_SPLIT;
    if (fork) {
      HIP_TRY(p, hipEventRecord(p->fork_ev, st));
      HIP_TRY(p, hipStreamWaitEvent(p->side, p->fork_ev, 0));
      if (fork2) HIP_TRY(p, hipStreamWaitEvent(p->side2, p->fork_ev, 0));
      si = p->side;
    }
    if (!p->tiles_int.empty()) {
      const int nt = (int)p->tiles_int.size();
      const unsigned gx = 8u * (unsigned)((nt + 7) / 8);
      TimedLaunch tl(p, fwd ? FWI_K_INTERIOR_ADJ : FWI_K_INTERIOR, si);
      if (fwd)
        interior_element_kernel<R, TX, TY, TZ, true, true><<<dim3(gx, 1), ETHREADS, 0, si>>>(
            G, p->d_tiles_int, nt, ns, Y, reg, lam(), mu(), res(), L.part, fwd, 3LL * G.si, gw, gacc(), L.gpart);
      else if (!mfma_interior(Y, nt, gx, si))
        interior_element_kernel<R, TX, TY, TZ, false, SRCLOOP><<<dim3(gx, SRCLOOP ? 1 : ns), ETHREADS, 0, si>>>(
            G, p->d_tiles_int, nt, ns, Y, reg, lam(), mu(), res(), L.part, nullptr, 0, 0.0, nullptr, L.gpart);
    }
    if (fork) HIP_TRY(p, hipEventRecord(p->join_ev, si));
    if (pml) {
      const int nt = (int)p->tiles_pml.size();
      const dim3 grid(8u * (unsigned)((nt + 7) / 8), SRCLOOP ? 1 : ns);
      TimedLaunch tl(p, adj ? FWI_K_PML_ADJ : FWI_K_PML, st);
      if (PMLFWI_PML_SPLIT) {
        // the two row types write disjoint rows: with three streams the
        // second part runs beside the first and the interior bricks
        if (adj) {
          launch_pml<PMLFWI_SPLIT_FIRST_ADJ>(adj, grid, nt, Y, reg, st);
          launch_pml<PML_ALL ^ PMLFWI_SPLIT_FIRST_ADJ>(adj, grid, nt, Y, reg, fork2 ? p->side2 : st);
        } else {
          launch_pml<PMLFWI_SPLIT_FIRST_FWD>(adj, grid, nt, Y, reg, st);
          launch_pml<PML_ALL ^ PMLFWI_SPLIT_FIRST_FWD>(adj, grid, nt, Y, reg, fork2 ? p->side2 : st);
        }
        if (fork2) HIP_TRY(p, hipEventRecord(p->join2_ev, p->side2));
      } else {
        launch_pml<PML_ALL>(adj, grid, nt, Y, reg, st);
      }
    }
    if (pml && pfwd) {
      // S-row terms of the gradient under the material extension; gacc slots
      // differ from the interior launch's, so the two may overlap
      const int nt = (int)p->tiles_pml.size();
      pml_gradient_kernel<R, TX, TY, TZ><<<8u * (unsigned)((nt + 7) / 8), ETHREADS, 0, st>>>(
          G, p->d_tiles_pml, nt, ns, Y, reg, pfwd, (long long)(9LL * G.sp), gw, gacc(), L.gpart);
    }
    if (fork) HIP_TRY(p, hipStreamWaitEvent(st, p->join_ev, 0));
    if (fork2) HIP_TRY(p, hipStreamWaitEvent(st, p->join2_ev, 0));
    HIP_TRY(p, hipGetLastError());
    return FWI_OK;
  }

  fwi_status nodal(int s, R* Yin, R* Yout, R* Xn, R* acc, const double* wav, int step, R* store,
                   R* pstore_ = nullptr) {
    static const double cA[4] = {1.0 / 6, 1.0 / 3, 1.0 / 3, 1.0 / 6};
    static const double cY[4] = {0.5, 0.5, 1.0, 0.0};
    static const int toff[4] = {0, 1, 1, 2};
    if (s == 0 && Yin != Xn) return fail(p, FWI_ERR_STATE, "internal: the first RK4 stage must start from Xn");
    const Geo& G = g();
    const double dt = p->prob.dt;
    NodalArgs<R> A{};
    A.Yin = Yin; A.Yout = Yout; A.Xn = Xn; A.acc = acc; A.res = res(); A.invMu = invm();
    A.part = L.part;
    A.reg = (long long)L.reg_elems;
    A.cA = R(cA[s] * dt); A.cY = R(cY[s] * dt);
    A.mode = s == 0 ? 0 : (s == 3 ? 2 : 1);
    if (wav && p->nload == 0) {
      A.src_node = p->d_src; A.src_dir = p->d_dir; A.wav = wav;
      A.wav_len = 2 * p->prob.nsteps + 1; A.wav_idx = 2 * step + toff[s];
    }
    A.store = store; A.store_stride = 3LL * G.si;
    A.pstore = store ? pstore_ : nullptr; A.pstore_stride = 9LL * G.sp;
    const long long rows = (long long)G.sn + G.n_pml;
    {
      TimedLaunch tl(p, FWI_K_NODAL, st);
      const int sm = !store ? 0 : (A.pstore ? 2 : 1);
      using K = void (*)(Geo, NodalArgs<R>);
      static const K table[3][3] = {
          {nodal_rk_kernel<R, 0, 0>, nodal_rk_kernel<R, 0, 1>, nodal_rk_kernel<R, 0, 2>},
          {nodal_rk_kernel<R, 1, 0>, nodal_rk_kernel<R, 1, 1>, nodal_rk_kernel<R, 1, 2>},
          {nodal_rk_kernel<R, 2, 0>, nodal_rk_kernel<R, 2, 1>, nodal_rk_kernel<R, 2, 2>}};
      const K kern = table[A.mode][sm];
      constexpr int NT = PMLFWI_NODAL_THREADS;
      if (PMLFWI_NODAL_ORDER == 2) {
        A.first = 0;
        A.last = G.sn;
        kern<<<dim3(blocks((size_t)G.sn, NT), p->nsrc), NT, 0, st>>>(G, A);
        A.first = G.sn;
        A.last = rows;
        kern<<<dim3(blocks((size_t)G.n_pml, NT), p->nsrc), NT, 0, st>>>(G, A);
      } else {
        const unsigned nb = (unsigned)blocks((size_t)rows, NT);
        A.first = 0;
        A.last = rows;
        A.rot = PMLFWI_NODAL_ORDER == 1 ? (unsigned)(G.sn / NT) % nb : 0u;
        kern<<<dim3(nb, p->nsrc), NT, 0, st>>>(G, A);
      }
    }
    if (wav && p->nload > 0) {
      load_kernel<R><<<blocks(p->nload, 128), 128, 0, st>>>(
          Yout, Xn, acc, (long long)L.reg_elems, G.sn, A.mode, cA[s] * dt, cY[s] * dt, invm(), p->nload,
          p->d_load_src, p->d_load_node, p->d_load_vec, wav, 2 * p->prob.nsteps + 1, 2 * step + toff[s]);
    }
    HIP_TRY(p, hipGetLastError());
    return FWI_OK;
  }

  // One RK4 step on (Xn, Ya, Yb, acc); `store_nl` >= 0 writes the stage
  // displacements of this step to store slot store_nl (and the next step's
  // first stage to store_nl+1 when store_next).
  fwi_status step(bool adj, int r0, int n, const double* wav, int store_nl, bool store_next,
                  int fwd_nl) {
    static const double bw[4] = {1.0 / 6, 1.0 / 3, 1.0 / 3, 1.0 / 6};
    R* Xn = reg(r0);
    R* Ya = reg(r0 + 1);
    R* Yb = reg(r0 + 2);
    R* acc = reg(r0 + 3);
    R* in = Xn;
    R* outs[4] = {Ya, Yb, Ya, nullptr};
    for (int s = 0; s < 4; ++s) {
      const R* fwd = fwd_nl >= 0 ? store(fwd_nl, 3 - s) : nullptr;
      const R* pfwd = fwd_nl >= 0 ? pstore(fwd_nl, 3 - s) : nullptr;
      fwi_status e = elements(adj, in, fwd, -bw[s] * p->prob.dt, false, pfwd);
      if (e != FWI_OK) return e;
      R* st_ = nullptr;
      R* pst_ = nullptr;
      if (store_nl >= 0) {
        if (s < 3) {
          st_ = store(store_nl, s + 1);
          pst_ = pstore(store_nl, s + 1);
        } else if (store_next) {
          st_ = store(store_nl + 1, 0);
          pst_ = pstore(store_nl + 1, 0);
        }
      }
      e = nodal(s, in, outs[s], Xn, acc, wav, n, st_, pst_);
      if (e != FWI_OK) return e;
      in = outs[s];
    }
    return FWI_OK;
  }

  fwi_status zero_regs(int r0, int nr) {
    fwi_status e = fill<R>(reg(r0), (size_t)nr * p->nsrc * L.reg_elems, R(0));
    if (e != FWI_OK) return e;
    return fill<R>(res(), (size_t)p->nsrc * L.part.per_src, R(0));
  }

  // Stage-store slot from a register: interior x1 displacement, and with the
  // full gradient the PML displacement fields (slot (nl, s)).
  fwi_status extract(const R* X, int nl, int s) {
    const Geo& G = g();
    extract_kernel<R><<<dim3(blocks(G.n_int, 256), p->nsrc), 256, 0, st>>>(G, X, (long long)L.reg_elems,
                                                                          store(nl, s), 3LL * G.si);
    if (R* ps = pstore(nl, s))
      pextract_kernel<R><<<dim3(blocks(G.n_pml, 256), p->nsrc), 256, 0, st>>>(G, X, (long long)L.reg_elems, ps,
                                                                             9LL * G.sp);
    HIP_TRY(p, hipGetLastError());
    return FWI_OK;
  }

  // keep = false: traces only, nothing kept for the adjoint.
  fwi_status forward(const double* rho, const double* lam_, const double* mu_, const double* wav,
                     double* traces, bool keep = true) {
    const fwi_problem& P = p->prob;
    fwi_status e;
    if ((e = setup(rho, lam_, mu_)) != FWI_OK) return e;
    if ((e = zero_regs(0, 4)) != FWI_OK) return e;
    const size_t tl = (size_t)P.nsrc * (P.nsteps + 1) * p->nrec * 3;
    if ((e = fill<double>(traces, tl, 0.0)) != FWI_OK) return e;
    keep = keep && P.ckpt_every >= 0;
    const bool keep_all = keep && P.ckpt_every == 0;
    const bool ckpts = keep && P.ckpt_every > 0;
    if (keep_all && (e = extract(reg(0), 0, 0)) != FWI_OK) return e;
    for (int n = 0; n < P.nsteps; ++n) {
      if (ckpts && n % P.ckpt_every == 0 && p->sched.fwd_slot[n / P.ckpt_every] >= 0)
        HIP_TRY(p, hipMemcpyAsync(ckpt(p->sched.fwd_slot[n / P.ckpt_every]), reg(0),
                                  (size_t)P.nsrc * L.reg_elems * L.es, hipMemcpyDeviceToDevice, st));
      if ((e = step(false, 0, n, wav, keep_all ? n : -1, n + 1 < P.nsteps, -1)) != FWI_OK)
        return e;
      if (p->nrec > 0) {
        receivers_kernel<R><<<dim3(blocks(p->nrec, 128), P.nsrc), 128, 0, st>>>(
            reg(0), (long long)L.reg_elems, g().sn, p->d_rec, p->nrec, traces, n + 1, P.nsteps);
        HIP_TRY(p, hipGetLastError());
      }
    }
    return FWI_OK;
  }

  fwi_status impulse(int r0, const double* resid, int n) {
    if (p->nrec == 0) return FWI_OK;
    const fwi_problem& P = p->prob;
    const double w = (n == 0 || n == P.nsteps) ? 0.5 : 1.0;
    impulse_kernel<R><<<dim3(blocks(p->nrec, 128), P.nsrc), 128, 0, st>>>(
        reg(r0), (long long)L.reg_elems, g().sn, invm(), p->d_rec, p->nrec, resid, n, P.nsteps, P.dt * w);
    HIP_TRY(p, hipGetLastError());
    return FWI_OK;
  }

  // Runs the checkpoint schedule; reverse(a, b) performs the adjoint steps
  // b-1 .. a once the stage store holds the segment [a, b) (slot n - a).
  template <typename F>
  fwi_status run_schedule(const double* wav, F&& reverse) {
    const fwi_problem& P = p->prob;
    const int k = P.ckpt_every;
    const size_t bytes = (size_t)P.nsrc * L.reg_elems * L.es;
    fwi_status e;
    for (const Act& act : p->sched.acts) {
      if (act.kind == ACT_LOAD) {
        if (act.a < 0) {
          if ((e = fill<R>(reg(0), (size_t)P.nsrc * L.reg_elems, R(0))) != FWI_OK) return e;
        } else {
          HIP_TRY(p, hipMemcpyAsync(reg(0), ckpt(act.a), bytes, hipMemcpyDeviceToDevice, st));
        }
      } else if (act.kind == ACT_SAVE) {
        HIP_TRY(p, hipMemcpyAsync(ckpt(act.a), reg(0), bytes, hipMemcpyDeviceToDevice, st));
      } else if (act.kind == ACT_ADVANCE) {
        for (int n = act.a * k; n < std::min(P.nsteps, act.b * k); ++n)
          if ((e = step(false, 0, n, wav, -1, false, -1)) != FWI_OK) return e;
      } else {
        const int a = act.a * k, b = std::min(P.nsteps, a + k);
        if ((e = extract(reg(0), 0, 0)) != FWI_OK) return e;
        for (int n = a; n < b; ++n)
          if ((e = step(false, 0, n, wav, n - a, n + 1 < b, -1)) != FWI_OK) return e;
        if ((e = reverse(a, b)) != FWI_OK) return e;
      }
    }
    return FWI_OK;
  }

  fwi_status adjoint(const double* rho, const double* lam_, const double* mu_, const double* wav,
                     const double* resid, double* gl, double* gm) {
    const fwi_problem& P = p->prob;
    const Geo& G = g();
    fwi_status e;
    if ((e = setup(rho, lam_, mu_)) != FWI_OK) return e;
    if ((e = fill<double>(gacc(), (size_t)L.gpart.per_src, 0.0)) != FWI_OK) return e;
    const bool keep_all = P.ckpt_every == 0;
    const int ra = keep_all ? 0 : 4;          // adjoint registers
    if ((e = zero_regs(ra, 4)) != FWI_OK) return e;
    if ((e = impulse(ra, resid, P.nsteps)) != FWI_OK) return e;
    auto reverse = [&](int a, int b) -> fwi_status {
      fwi_status e2;
      for (int n = b - 1; n >= a; --n) {
        if ((e2 = step(true, ra, n, nullptr, -1, false, n - a)) != FWI_OK) return e2;
        if (n > 0 && (e2 = impulse(ra, resid, n)) != FWI_OK) return e2;
      }
      return FWI_OK;
    };
    if (keep_all) {
      if ((e = reverse(0, P.nsteps)) != FWI_OK) return e;
    } else if ((e = run_schedule(wav, reverse)) != FWI_OK) {
      return e;
    }
    if (p->prob.grad_full)
      gradient_reduce_full_kernel<<<blocks(G.n_int, 256), 256, 0, st>>>(G, gacc(), L.gpart, gl, gm);
    else
      gradient_reduce_kernel<<<blocks(G.n_int, 256), 256, 0, st>>>(G, gacc(), L.gpart, gl, gm);
    HIP_TRY(p, hipGetLastError());
    return FWI_OK;
  }

  // The paper's reverse-time RK4 of the adjoint problem (App. B): from
  // y(T) = 0, step n (t_{n+1} -> t_n) is classical RK4 on the transposed
  // operator for z = (y0, -y1, y2) with the receiver residual as forcing at
  // the stage times (r_{n+1}, the mean of r_{n+1} and r_n twice, r_n); the
  // gradient (C.1f)-(C.1g) is the trapezoid rule over the step states:
  // g += dt w_n z1^T (dK_RD/dm) u^n.
  fwi_status adjoint_appb(const double* rho, const double* lam_, const double* mu_, const double* wav,
                          const double* resid, double* gl, double* gm) {
    static const double cA[4] = {1.0 / 6, 1.0 / 3, 1.0 / 3, 1.0 / 6};
    static const double cY[4] = {0.5, 0.5, 1.0, 0.0};
    const fwi_problem& P = p->prob;
    const Geo& G = g();
    const double dt = P.dt;
    fwi_status e;
    if ((e = setup(rho, lam_, mu_)) != FWI_OK) return e;
    if ((e = fill<double>(gacc(), (size_t)L.gpart.per_src, 0.0)) != FWI_OK) return e;
    const bool keep_all = P.ckpt_every == 0;
    const int ra = keep_all ? 0 : 4;
    if ((e = zero_regs(ra, 4)) != FWI_OK) return e;
    auto reverse = [&](int a, int b) -> fwi_status {
      fwi_status e2 = FWI_OK;
      for (int n = b - 1; n >= a; --n) {
        R* Xn = reg(ra);
        R* outs[4] = {reg(ra + 1), reg(ra + 2), reg(ra + 1), nullptr};
        R* in = Xn;
        for (int s = 0; s < 4; ++s) {
          if ((e2 = elements(true, in, nullptr, 0.0)) != FWI_OK) return e2;
          if ((e2 = nodal(s, in, outs[s], Xn, reg(ra + 3), nullptr, n, nullptr)) != FWI_OK) return e2;
          if (p->nrec > 0) {
            const int mode = s == 0 ? 0 : (s == 3 ? 2 : 1);
            const double ah = s == 0 ? 1.0 : (s == 3 ? 0.0 : 0.5), al = 1.0 - ah;
            appb_force_kernel<R><<<dim3(blocks(p->nrec, 128), P.nsrc), 128, 0, st>>>(
                outs[s], Xn, reg(ra + 3), (long long)L.reg_elems, G.sn, mode, cA[s] * dt, cY[s] * dt, invm(),
                p->d_rec, p->nrec, resid, n + 1, n, ah, al, P.nsteps);
            HIP_TRY(p, hipGetLastError());
          }
          in = outs[s];
        }
        const double w = (n == 0 || n == P.nsteps) ? 0.5 : 1.0;
        if ((e2 = elements(true, Xn, store(n - a, 0), dt * w, true)) != FWI_OK) return e2;
      }
      return e2;
    };
    if (keep_all) {
      if ((e = reverse(0, P.nsteps)) != FWI_OK) return e;
    } else if ((e = run_schedule(wav, reverse)) != FWI_OK) {
      return e;
    }
    gradient_reduce_kernel<<<blocks(G.n_int, 256), 256, 0, st>>>(G, gacc(), L.gpart, gl, gm);
    HIP_TRY(p, hipGetLastError());
    return FWI_OK;
  }

  // Largest eigenvalue of M_RD^{-1} K_RD by `iters` power iterations on the
  // first source's registers 0 and 1 (overwritten); the result (running
  // maximum of the Rayleigh quotients) is left in p->d_info[7].
  fwi_status power_omega(const double* rho, const double* lam_, const double* mu_, int iters) {
    const Geo& G = g();
    fwi_status e;
    if ((e = setup(rho, lam_, mu_)) != FWI_OK) return e;
    if ((e = zero_regs(0, 2)) != FWI_OK) return e;
    double* state = p->d_info + 5;
    power_init_kernel<R><<<blocks(G.n_nodes, 256), 256, 0, st>>>(G, reg(0), state);
    HIP_TRY(p, hipGetLastError());
    const int nb = (int)std::min<size_t>(blocks(G.n_nodes, 256), MISFIT_BLOCKS / 3);
    for (int it = 0; it < iters; ++it) {
      R* X = reg(it & 1);
      R* Y = reg((it + 1) & 1);
      if ((e = elements(false, X, nullptr, 0.0, true)) != FWI_OK) return e;
      power_step_kernel<R><<<nb, 256, 0, st>>>(G, X, Y, res(), L.part, rho, it == 0, state, p->d_partials);
      power_reduce_kernel<<<1, 256, 0, st>>>(p->d_partials, nb, state);
      HIP_TRY(p, hipGetLastError());
    }
    return FWI_OK;
  }

  fwi_status apply(int which, const double* rho, const double* lam_, const double* mu_, const double* x0,
                   const double* x1, const double* x2, double* out) {
    const Geo& G = g();
    fwi_status e;
    if ((e = setup(rho, lam_, mu_)) != FWI_OK) return e;
    if ((e = zero_regs(0, 1)) != FWI_OK) return e;
    const double* xs[3] = {x0, x1, x2};
    for (int s = 0; s < 3; ++s) {
      pack_kernel<R><<<dim3(blocks(G.n_nodes, 256), p->nsrc), 256, 0, st>>>(G, xs[s], reg(0), (long long)L.reg_elems, s);
      HIP_TRY(p, hipGetLastError());
    }
    if ((e = elements(which == 1, reg(0), nullptr, 0.0)) != FWI_OK) return e;
    accel_kernel<R><<<dim3(blocks(G.n_nodes, 256), p->nsrc), 256, 0, st>>>(
        G, reg(0), (long long)L.reg_elems, res(), L.part, invm(), out);
    HIP_TRY(p, hipGetLastError());
    return FWI_OK;
  }
};

// Model check before a solve: one small kernel, a copy of 5 doubles and a
// stream synchronization.  info: 6 host doubles (see fwi_check_model).
// With a workspace, a time step above the brick-by-brick bound is checked
// again against a power-iteration estimate of the largest frequency of the
// interior operator (that bound overestimates it by about 1.2x, enough to
// reject the paper's own Sec. 4.1 step): accepted when dt omega_est stays 2 %
// below the RK4 limit 2 sqrt(2).  info[4], info[5] then hold the estimate.
constexpr int POWER_ITERS = 150;
constexpr double POWER_MARGIN = 1.02;

template <typename F>
fwi_status dispatch(fwi_plan* p, hipStream_t st, void* ws, F&& f, bool keep = true);

fwi_status check_model(fwi_plan* p, hipStream_t st, const double* rho, const double* lam, const double* mu,
                       double* info, const char* who, void* ws = nullptr, bool keep = true) {
  model_check_kernel<<<1, 1024, 0, st>>>(p->g, rho, lam, mu, p->c_lam, p->c_mu, p->d_info);
  hipError_t e = hipGetLastError();
  if (e == hipSuccess) e = hipMemcpyAsync(p->h_info, p->d_info, 5 * sizeof(double), hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) return fail(p, FWI_ERR_HIP, std::string(who) + ": model check: " + hipGetErrorString(e));
  const double* v = p->h_info;
  // omega_max^2 <= max over bricks of the brick bound; the unit reference brick
  // has edge 2, so a brick of edge h scales it by (2/h)^2
  const double h = p->g.h;
  const double wmax = std::sqrt(v[4] * 4.0 / (h * h));
  for (int k = 0; k < 4; ++k) info[k] = v[k];
  info[4] = wmax;
  info[5] = wmax > 0 ? 2.0 * std::sqrt(2.0) / wmax : HUGE_VAL;
  char msg[320];
  if (!(v[0] > 0.0) || !(v[1] > 0.0) || !(v[2] > 0.0)) {
    std::snprintf(msg, sizeof(msg), "%s: rho, mu and 3 lam + 2 mu must be positive (min rho %g, min mu %g, "
                  "min 3 lam + 2 mu %g)", who, v[0], v[1], v[2]);
    return fail(p, FWI_ERR_ARG, msg);
  }
  if (p->prob.dt <= info[5]) return FWI_OK;
  if (ws) {
    fwi_status s = dispatch(p, st, ws, [&](auto& r) { return r.power_omega(rho, lam, mu, POWER_ITERS); }, keep);
    if (s != FWI_OK) return s;
    e = hipMemcpyAsync(p->h_info + 5, p->d_info + 5, 3 * sizeof(double), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return fail(p, FWI_ERR_HIP, std::string(who) + ": power iteration: " + hipGetErrorString(e));
    const double west = std::sqrt(std::max(p->h_info[7], 0.0));
    info[4] = west;
    info[5] = west > 0 ? 2.0 * std::sqrt(2.0) / (POWER_MARGIN * west) : HUGE_VAL;
    if (p->prob.dt <= info[5]) return FWI_OK;
    std::snprintf(msg, sizeof(msg), "%s: dt %.6g s above the RK4 stability bound %.6g s (power-iteration estimate "
                  "of omega_max %.6g 1/s, brick bound %.6g 1/s)", who, p->prob.dt, info[5], west, wmax);
    return fail(p, FWI_ERR_UNSTABLE, msg);
  }
  std::snprintf(msg, sizeof(msg), "%s: dt %.6g s above the RK4 stability bound %.6g s (omega_max bound %.6g 1/s)",
                who, p->prob.dt, info[5], wmax);
  return fail(p, FWI_ERR_UNSTABLE, msg);
}

template <typename F>
fwi_status dispatch(fwi_plan* p, hipStream_t st, void* ws, F&& f, bool keep) {
  Layout L = layout(p->prob, p->g, keep);
  if (p->prob.precision != FWI_FP64) {
    Run<float> r{p, st, L, (char*)ws};
    return f(r);
  }
  Run<double> r{p, st, L, (char*)ws};
  return f(r);
}

}  // namespace

// ------------------------------------------------ fixed scratch (no allocation)
// Workspace of fwi_forward_noalloc: a file-scope device array, one copy per
// GPU, held until the process ends.  Host code never uses the array's name as
// an address: the device address is looked up once per device
// (hipGetSymbolAddress, at fwi_plan_create with that device current) and
// kept in g_scratch_addr and in every plan made on that device.
constexpr size_t NOALLOC_SCRATCH_BYTES = size_t(64) << 20;
static __device__ __align__(256) unsigned char scratch[NOALLOC_SCRATCH_BYTES];

namespace {
constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void* g_scratch_addr[MAX_DEVICES] = {};

// Device address of the scratch array on `device` (which must be current).
hipError_t scratch_address(int device, void** out) {
  *out = nullptr;
  if (device < 0 || device >= MAX_DEVICES) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_addr[device]) {
    void* ptr = nullptr;
    hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!ptr) return hipErrorInvalidSymbol;
    g_scratch_addr[device] = ptr;
  }
  *out = g_scratch_addr[device];
  return hipSuccess;
}
}  // namespace

// ====================================================================== C ABI
extern "C" {

fwi_status fwi_query(const fwi_problem* prob, fwi_sizes* out) {
  if (!prob || !out) return FWI_ERR_ARG;
  fwi_status v = validate(prob);
  if (v != FWI_OK) return v;
  const Geo g = make_geo(*prob);
  const Layout L = layout(*prob, g);
  const int64_t free_nodes = (int64_t)(g.NX - 2) * (g.NY - 2) * (g.NZ - 1);
  const int64_t dir_nodes = (int64_t)g.n_nodes - free_nodes;
  out->n_nodes = g.n_nodes;
  out->n_int_nodes = g.n_int;
  out->n_pml_nodes = g.n_pml;
  out->n_state = 3 * free_nodes + 6 * (int64_t)g.n_pml;
  out->n_hist = 3 * ((int64_t)g.n_pml - dir_nodes) + 6 * (int64_t)g.n_pml;
  out->trace_len = (int64_t)prob->nsrc * (prob->nsteps + 1) * prob->nrec * 3;
  out->workspace_bytes = (int64_t)L.total;
  out->register_bytes = (int64_t)(prob->nsrc * L.reg_elems * L.es);
  out->tile[0] = TX;
  out->tile[1] = TY;
  out->tile[2] = TZ;
  const int64_t nx = count_faces(*prob, g, 0), ny = count_faces(*prob, g, 1), nz = count_faces(*prob, g, 2);
  const int64_t ix = (g.ex + TX - 1) / TX, iy = (g.ey + TY - 1) / TY, iz = (g.ez + TZ - 1) / TZ;
  out->tiles_interior = ix * iy * iz;
  out->tiles_pml = nx * ny * nz - ix * iy * iz;
  out->element_threads = ETHREADS;
  const Schedule S = make_schedule(*prob);
  out->ckpt_states = L.nckpt;
  out->schedule_advances = S.advances;
  out->adjoint_forward_steps = S.adjoint_steps;
  return FWI_OK;
}

fwi_status fwi_plan_create(const fwi_problem* prob, const int32_t* src_node, const double* src_dir,
                           const int32_t* rec_node, fwi_plan** out) {
  if (!out) return FWI_ERR_ARG;
  *out = nullptr;
  fwi_status v = validate(prob);
  if (v != FWI_OK) return v;
  if (!src_node || !src_dir || (prob->nrec > 0 && !rec_node)) return FWI_ERR_ARG;
  fwi_plan* p = new (std::nothrow) fwi_plan();
  if (!p) return FWI_ERR_NOMEM;
  p->prob = *prob;
  p->g = make_geo(*prob);
  p->nsrc = prob->nsrc;
  p->nrec = prob->nrec;
  const Geo& g = p->g;
  auto bad_node = [&](int32_t id) {
    if (id < 0 || id >= g.n_nodes) return true;
    const int k = id / g.plane, r = id - k * g.plane, j = r / g.NX, i = r - j * g.NX;
    return is_dirichlet(g, i, j, k);
  };
  for (int s = 0; s < prob->nsrc; ++s)
    if (bad_node(src_node[s])) { delete p; return FWI_ERR_ARG; }
  for (int r = 0; r < prob->nrec; ++r)
    if (bad_node(rec_node[r])) { delete p; return FWI_ERR_ARG; }
  build_tiles(p);
  p->sched = make_schedule(*prob);
  p->c_lam = reference_eigen(1.0, 0.0);
  p->c_mu = reference_eigen(0.0, 1.0);
  auto up = [&](void** dst, const void* src, size_t bytes) -> hipError_t {
    if (bytes == 0) return hipSuccess;
    hipError_t e = hipMalloc(dst, bytes);
    if (e != hipSuccess) return e;
    return hipMemcpy(*dst, src, bytes, hipMemcpyHostToDevice);
  };
  hipError_t e = hipSuccess;
  const char* what = "";
  auto step = [&](const char* name, void** dst, const void* src, size_t bytes) {
    if (e == hipSuccess) {
      e = up(dst, src, bytes);
      what = name;
    }
  };
  step("brick tiles", (void**)&p->d_tiles_int, p->tiles_int.data(), p->tiles_int.size() * sizeof(Tile));
  step("PML tiles", (void**)&p->d_tiles_pml, p->tiles_pml.data(), p->tiles_pml.size() * sizeof(Tile));
  step("source nodes", (void**)&p->d_src, src_node, prob->nsrc * sizeof(int32_t));
  step("source directions", (void**)&p->d_dir, src_dir, prob->nsrc * 3 * sizeof(double));
  step("receiver nodes", (void**)&p->d_rec, rec_node, prob->nrec * sizeof(int32_t));
  step("axis tables", (void**)&p->d_tab, p->tab.data(), p->tab.size() * sizeof(double));
  step("face ordinals", (void**)&p->d_fo, p->fo.data(), p->fo.size() * sizeof(int));
  const double zeros[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  step("model-check buffer", (void**)&p->d_info, zeros, sizeof(zeros));
  if (e == hipSuccess) {
    what = "misfit partial sums";
    e = hipMalloc((void**)&p->d_partials, MISFIT_BLOCKS * sizeof(double));
  }
  // the stream the interior bricks run on beside the PML bricks, and its
  // fork / join events (created here so that the solves allocate nothing)
  if (e == hipSuccess) {
    what = "side stream";
    e = hipStreamCreateWithFlags(&p->side, hipStreamNonBlocking);
  }
  if (e == hipSuccess) e = hipEventCreateWithFlags(&p->fork_ev, hipEventDisableTiming);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&p->join_ev, hipEventDisableTiming);
  if (e == hipSuccess && PMLFWI_CONCURRENT == 2) {
    e = hipStreamCreateWithFlags(&p->side2, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&p->join2_ev, hipEventDisableTiming);
  }
  if (e == hipSuccess) {
    what = "pinned model-check result";
    e = hipHostMalloc((void**)&p->h_info, 8 * sizeof(double), hipHostMallocDefault);
  }
  if (e == hipSuccess) {
    what = "device id";
    e = hipGetDevice(&p->device);
  }
  if (e == hipSuccess) {
    what = "address of the fixed scratch array";
    e = scratch_address(p->device, &p->scratch);
  }
  p->g.tab = p->d_tab;
  p->g.fo = p->d_fo;
  if (e != hipSuccess) {
    g_plan_err = std::string("fwi_plan_create: upload of the ") + what + ": " + hipGetErrorString(e);
    fwi_plan_destroy(p);
    return FWI_ERR_HIP;
  }
  *out = p;
  return FWI_OK;
}

fwi_status fwi_plan_set_loads(fwi_plan* p, int32_t nload, const int32_t* load_src, const int32_t* load_node,
                              const double* load_vec) {
  if (!p) return FWI_ERR_ARG;
  if (nload < 0 || (nload > 0 && (!load_src || !load_node || !load_vec)))
    return fail(p, FWI_ERR_ARG, "fwi_plan_set_loads: bad count or null pointer");
  const Geo& g = p->g;
  // merge entries of the same (source, node): the load kernel then writes each
  // register entry from one thread
  std::vector<std::pair<long long, int>> key(nload);
  for (int e = 0; e < nload; ++e) {
    const int s = load_src[e], id = load_node[e];
    if (s < 0 || s >= p->nsrc) return fail(p, FWI_ERR_ARG, "fwi_plan_set_loads: source index out of range");
    if (id < 0 || id >= g.n_nodes) return fail(p, FWI_ERR_ARG, "fwi_plan_set_loads: node id out of range");
    const int k = id / g.plane, r = id - k * g.plane, j = r / g.NX, i = r - j * g.NX;
    if (is_dirichlet(g, i, j, k)) return fail(p, FWI_ERR_ARG, "fwi_plan_set_loads: load on a Dirichlet node");
    key[e] = {(long long)s * g.n_nodes + id, e};
  }
  std::sort(key.begin(), key.end());
  std::vector<int32_t> hs, hn;
  std::vector<double> hv;
  for (int e = 0; e < nload; ++e) {
    const int o = key[e].second;
    if (e == 0 || key[e].first != key[e - 1].first) {
      hs.push_back(load_src[o]);
      hn.push_back(load_node[o]);
      hv.insert(hv.end(), {load_vec[3 * o], load_vec[3 * o + 1], load_vec[3 * o + 2]});
    } else {
      for (int d = 0; d < 3; ++d) hv[hv.size() - 3 + d] += load_vec[3 * o + d];
    }
  }
  HIP_TRY(p, hipDeviceSynchronize());   // the old tables may still be in use
  (void)hipFree(p->d_load_src);
  (void)hipFree(p->d_load_node);
  (void)hipFree(p->d_load_vec);
  p->d_load_src = p->d_load_node = nullptr;
  p->d_load_vec = nullptr;
  p->nload = 0;
  const int n = (int)hs.size();
  if (n == 0) return FWI_OK;
  HIP_TRY(p, hipMalloc((void**)&p->d_load_src, n * sizeof(int32_t)));
  HIP_TRY(p, hipMalloc((void**)&p->d_load_node, n * sizeof(int32_t)));
  HIP_TRY(p, hipMalloc((void**)&p->d_load_vec, 3 * n * sizeof(double)));
  HIP_TRY(p, hipMemcpy(p->d_load_src, hs.data(), n * sizeof(int32_t), hipMemcpyHostToDevice));
  HIP_TRY(p, hipMemcpy(p->d_load_node, hn.data(), n * sizeof(int32_t), hipMemcpyHostToDevice));
  HIP_TRY(p, hipMemcpy(p->d_load_vec, hv.data(), 3 * n * sizeof(double), hipMemcpyHostToDevice));
  p->nload = n;
  return FWI_OK;
}

fwi_status fwi_surface_traction(const fwi_problem* prob, double xmin, double xmax, double ymin, double ymax,
                                int32_t cap, int32_t* node, double* weight, int32_t* count) {
  if (!prob || !count || cap < 0 || (cap > 0 && (!node || !weight))) return FWI_ERR_ARG;
  fwi_status v = validate(prob);
  if (v != FWI_OK) return v;
  if (!(xmin <= xmax) || !(ymin <= ymax)) return FWI_ERR_ARG;
  const Geo g = make_geo(*prob);
  const double h = g.h;
  // one-dimensional weights: sum over the surface-face edges [a, a + h] inside
  // [lo, hi] of the LGL weight of the node times h/2
  auto axis = [&](double lo, double hi, double x0, int n, std::vector<double>& w) {
    w.assign(n, 0.0);
    for (int e = 0; 2 * e + 2 < n; ++e) {
      const double a = x0 + e * h, b = a + h;
      if (a < lo - 1e-9 * h || b > hi + 1e-9 * h) continue;
      w[2 * e] += h / 6.0;
      w[2 * e + 1] += 2.0 * h / 3.0;
      w[2 * e + 2] += h / 6.0;
    }
  };
  std::vector<double> wx, wy;
  axis(xmin, xmax, g.x0, g.NX, wx);
  axis(ymin, ymax, g.y0, g.NY, wy);
  int32_t c = 0;
  const int k = g.NZ - 1;
  for (int j = 0; j < g.NY; ++j)
    for (int i = 0; i < g.NX; ++i) {
      const double w = wx[i] * wy[j];
      if (w == 0.0 || is_dirichlet(g, i, j, k)) continue;
      if (c < cap) {
        node[c] = i + g.NX * (j + g.NY * k);
        weight[c] = w;
      }
      ++c;
    }
  *count = c;
  return c <= cap ? FWI_OK : FWI_ERR_SHAPE;
}

fwi_status fwi_timing_enable(fwi_plan* p, int stride) {
  if (!p || stride < 0) return FWI_ERR_ARG;
  p->tstride = stride;
  for (int c = 0; c < FWI_K_NCLASS; ++c) {
    p->launches[c] = 0;
    p->ev_used[c] = 0;
  }
  return FWI_OK;
}

fwi_status fwi_timing_read(fwi_plan* p, int cls, double* mean_ms, int64_t* samples, int64_t* launches) {
  if (!p || cls < 0 || cls >= FWI_K_NCLASS || !mean_ms || !samples || !launches) return FWI_ERR_ARG;
  double tot = 0.0;
  for (size_t i = 0; i < p->ev_used[cls]; ++i) {
    auto& e = p->ev[cls][i];
    HIP_TRY(p, hipEventSynchronize(e.second));
    float ms = 0.f;
    HIP_TRY(p, hipEventElapsedTime(&ms, e.first, e.second));
    tot += ms;
  }
  *samples = (int64_t)p->ev_used[cls];
  *launches = p->launches[cls];
  *mean_ms = p->ev_used[cls] ? tot / p->ev_used[cls] : 0.0;
  return FWI_OK;
}

fwi_status fwi_plan_destroy(fwi_plan* p) {
  if (!p) return FWI_ERR_ARG;
  for (auto& v : p->ev)
    for (auto& e : v) {
      (void)hipEventDestroy(e.first);
      (void)hipEventDestroy(e.second);
    }
  if (p->side) (void)hipStreamSynchronize(p->side);
  if (p->fork_ev) (void)hipEventDestroy(p->fork_ev);
  if (p->join_ev) (void)hipEventDestroy(p->join_ev);
  if (p->side) (void)hipStreamDestroy(p->side);
  if (p->side2) (void)hipStreamSynchronize(p->side2);
  if (p->join2_ev) (void)hipEventDestroy(p->join2_ev);
  if (p->side2) (void)hipStreamDestroy(p->side2);
  (void)hipFree(p->d_tiles_int);
  (void)hipFree(p->d_tiles_pml);
  (void)hipFree(p->d_src);
  (void)hipFree(p->d_dir);
  (void)hipFree(p->d_rec);
  (void)hipFree(p->d_load_src);
  (void)hipFree(p->d_load_node);
  (void)hipFree(p->d_load_vec);
  (void)hipFree(p->d_tab);
  (void)hipFree(p->d_fo);
  (void)hipFree(p->d_info);
  (void)hipFree(p->d_partials);
  if (p->h_info) (void)hipHostFree(p->h_info);
  delete p;
  return FWI_OK;
}

fwi_status fwi_forward(fwi_plan* p, void* stream, const double* rho, const double* lam, const double* mu,
                       const double* wavelet, void* workspace, double* traces) {
  if (!p) return FWI_ERR_ARG;
  if (!rho || !lam || !mu || !wavelet || !workspace || (p->nrec > 0 && !traces))
    return fail(p, FWI_ERR_ARG, "fwi_forward: null pointer");
  p->fwd_ws = nullptr;
  double info[6];
  if (fwi_status c = check_model(p, (hipStream_t)stream, rho, lam, mu, info, "fwi_forward", workspace); c != FWI_OK)
    return c;
  fwi_status s = dispatch(p, (hipStream_t)stream, workspace,
                          [&](auto& r) { return r.forward(rho, lam, mu, wavelet, traces); });
  if (s == FWI_OK) p->fwd_ws = workspace;
  return s;
}

fwi_status fwi_forward_noalloc(fwi_plan* p, void* stream, const double* rho, const double* lam, const double* mu,
                               const double* wavelet, double* traces) {
  if (!p) return FWI_ERR_ARG;
  if (!rho || !lam || !mu || !wavelet || (p->nrec > 0 && !traces))
    return fail(p, FWI_ERR_ARG, "fwi_forward_noalloc: null pointer");
  if (!p->scratch) return fail(p, FWI_ERR_HIP, "fwi_forward_noalloc: no scratch address for this device");
  int dev = -1;
  HIP_TRY(p, hipGetDevice(&dev));
  if (dev != p->device) return fail(p, FWI_ERR_ARG, "fwi_forward_noalloc: the plan belongs to another device");
  const size_t need = layout(p->prob, p->g, false).total;
  if (need > NOALLOC_SCRATCH_BYTES) {
    char msg[200];
    std::snprintf(msg, sizeof(msg), "fwi_forward_noalloc: this problem needs %zu bytes of workspace, more than "
                  "the fixed scratch of %zu bytes", need, NOALLOC_SCRATCH_BYTES);
    return fail(p, FWI_ERR_ARG, msg);
  }
  double info[6];
  if (fwi_status c = check_model(p, (hipStream_t)stream, rho, lam, mu, info, "fwi_forward_noalloc", p->scratch,
                                 false); c != FWI_OK)
    return c;
  // the forward registers in the plan's workspace (if any) are not touched, so
  // an fwi_adjoint_gradient after this call still sees the last fwi_forward
  const int tstride = p->tstride;   // sampled timing would create events
  p->tstride = 0;
  fwi_status s = dispatch(p, (hipStream_t)stream, p->scratch,
                          [&](auto& r) { return r.forward(rho, lam, mu, wavelet, traces, false); }, false);
  p->tstride = tstride;
  return s;
}

fwi_status fwi_misfit(fwi_plan* p, void* stream, const double* traces, const double* observed, double* residual,
                      double* J) {
  if (!p) return FWI_ERR_ARG;
  if (!traces || !observed || !residual || !J) return fail(p, FWI_ERR_ARG, "fwi_misfit: null pointer");
  hipStream_t st = (hipStream_t)stream;
  const long long n = (long long)p->nsrc * (p->prob.nsteps + 1) * p->nrec * 3;
  if (n == 0) {
    fill_kernel<double><<<1, 32, 0, st>>>(J, 1, 0.0);
  } else {
    const int nb = (int)std::min<long long>((n + 255) / 256, MISFIT_BLOCKS);
    misfit_kernel<<<nb, 256, 0, st>>>(traces, observed, residual, n, p->nrec * 3, p->prob.nsteps, p->d_partials);
    misfit_final_kernel<<<1, 256, 0, st>>>(p->d_partials, nb, 0.5 * p->prob.dt, J);
  }
  HIP_TRY(p, hipGetLastError());
  return FWI_OK;
}

fwi_status fwi_adjoint_gradient(fwi_plan* p, void* stream, const double* rho, const double* lam,
                                const double* mu, const double* wavelet, const double* residual,
                                void* workspace, double* g_lam, double* g_mu) {
  if (!p) return FWI_ERR_ARG;
  if (!rho || !lam || !mu || !wavelet || !workspace || !g_lam || !g_mu || (p->nrec > 0 && !residual))
    return fail(p, FWI_ERR_ARG, "fwi_adjoint_gradient: null pointer");
  if (p->prob.ckpt_every < 0)
    return fail(p, FWI_ERR_STATE, "fwi_adjoint_gradient: forward-only plan (ckpt_every < 0) keeps nothing for an adjoint");
  if (p->fwd_ws != workspace)
    return fail(p, FWI_ERR_STATE, "fwi_adjoint_gradient: no fwi_forward on this workspace");
  double info[6];
  if (fwi_status c = check_model(p, (hipStream_t)stream, rho, lam, mu, info, "fwi_adjoint_gradient", workspace); c != FWI_OK)
    return c;
  return dispatch(p, (hipStream_t)stream, workspace,
                  [&](auto& r) { return r.adjoint(rho, lam, mu, wavelet, residual, g_lam, g_mu); });
}

fwi_status fwi_adjoint_gradient_appb(fwi_plan* p, void* stream, const double* rho, const double* lam,
                                     const double* mu, const double* wavelet, const double* residual,
                                     void* workspace, double* g_lam, double* g_mu) {
  if (!p) return FWI_ERR_ARG;
  if (!rho || !lam || !mu || !wavelet || !workspace || !g_lam || !g_mu || (p->nrec > 0 && !residual))
    return fail(p, FWI_ERR_ARG, "fwi_adjoint_gradient_appb: null pointer");
  if (p->prob.grad_full)
    return fail(p, FWI_ERR_ARG, "fwi_adjoint_gradient_appb: the full gradient (grad_full = 1) is built for the "
                                "exact adjoint only");
  if (p->prob.ckpt_every < 0)
    return fail(p, FWI_ERR_STATE, "fwi_adjoint_gradient_appb: forward-only plan (ckpt_every < 0) keeps nothing for an adjoint");
  if (p->fwd_ws != workspace)
    return fail(p, FWI_ERR_STATE, "fwi_adjoint_gradient_appb: no fwi_forward on this workspace");
  double info[6];
  if (fwi_status c = check_model(p, (hipStream_t)stream, rho, lam, mu, info, "fwi_adjoint_gradient_appb", workspace); c != FWI_OK)
    return c;
  return dispatch(p, (hipStream_t)stream, workspace,
                  [&](auto& r) { return r.adjoint_appb(rho, lam, mu, wavelet, residual, g_lam, g_mu); });
}

fwi_status fwi_apply_operator(fwi_plan* p, void* stream, int which, const double* rho, const double* lam,
                              const double* mu, const double* x0, const double* x1, const double* x2,
                              void* workspace, double* out) {
  if (!p) return FWI_ERR_ARG;
  if (which != 0 && which != 1) return fail(p, FWI_ERR_ARG, "fwi_apply_operator: which must be 0 or 1");
  if (!rho || !lam || !mu || !x0 || !x1 || !x2 || !workspace || !out)
    return fail(p, FWI_ERR_ARG, "fwi_apply_operator: null pointer");
  p->fwd_ws = nullptr;   // the hook reuses the forward registers
  return dispatch(p, (hipStream_t)stream, workspace,
                  [&](auto& r) { return r.apply(which, rho, lam, mu, x0, x1, x2, out); });
}

fwi_status fwi_regularization(fwi_plan* p, void* stream, int kind, double eps, const double* field,
                              double* value, double* grad) {
  if (!p) return FWI_ERR_ARG;
  if (kind != FWI_REG_TIKHONOV && kind != FWI_REG_TV)
    return fail(p, FWI_ERR_ARG, "fwi_regularization: kind must be FWI_REG_TIKHONOV or FWI_REG_TV");
  if (kind == FWI_REG_TV && !(eps > 0)) return fail(p, FWI_ERR_ARG, "fwi_regularization: TV needs eps > 0");
  if (!field || (!value && !grad)) return fail(p, FWI_ERR_ARG, "fwi_regularization: null pointer");
  hipStream_t st = (hipStream_t)stream;
  const Geo& G = p->g;
  const int k = kind == FWI_REG_TIKHONOV ? REG_TN : REG_TV;
  if (grad) reg_gradient_kernel<<<blocks(G.n_int, 256), 256, 0, st>>>(G, k, eps, field, grad);
  if (value) reg_value_kernel<<<1, 1024, 0, st>>>(G, k, eps, field, value);
  HIP_TRY(p, hipGetLastError());
  return FWI_OK;
}

fwi_status fwi_material_mass(fwi_plan* p, void* stream, double* mdiag) {
  if (!p) return FWI_ERR_ARG;
  if (!mdiag) return fail(p, FWI_ERR_ARG, "fwi_material_mass: null pointer");
  material_mass_kernel<<<blocks(p->g.n_int, 256), 256, 0, (hipStream_t)stream>>>(p->g, mdiag);
  HIP_TRY(p, hipGetLastError());
  return FWI_OK;
}

fwi_status fwi_gradient_finalize(fwi_plan* p, void* stream, const double* g_mis, const double* g_reg, double R,
                                 double* g) {
  if (!p) return FWI_ERR_ARG;
  if (!g_mis || !g || (R != 0.0 && !g_reg)) return fail(p, FWI_ERR_ARG, "fwi_gradient_finalize: null pointer");
  gradient_finalize_kernel<<<blocks(p->g.n_int, 256), 256, 0, (hipStream_t)stream>>>(p->g, g_mis, g_reg, R, g);
  HIP_TRY(p, hipGetLastError());
  return FWI_OK;
}

fwi_status fwi_check_model(fwi_plan* p, void* stream, const double* rho, const double* lam, const double* mu,
                           double* info) {
  if (!p) return FWI_ERR_ARG;
  if (!rho || !lam || !mu || !info) return fail(p, FWI_ERR_ARG, "fwi_check_model: null pointer");
  return check_model(p, (hipStream_t)stream, rho, lam, mu, info, "fwi_check_model");
}

fwi_status fwi_dot(void* stream, int64_t n, const double* a, const double* b, const double* w, double* out) {
  if (n < 0 || !out || (n > 0 && (!a || !b))) return FWI_ERR_ARG;
  dot_kernel<<<1, 1024, 0, (hipStream_t)stream>>>((long long)n, a, b, w, out);
  return hipGetLastError() == hipSuccess ? FWI_OK : FWI_ERR_HIP;
}

fwi_status fwi_axpby(void* stream, int64_t n, double alpha, const double* x, double beta, const double* y,
                     double* out) {
  if (n < 0 || (n > 0 && (!x || !out || (beta != 0.0 && !y)))) return FWI_ERR_ARG;
  if (n == 0) return FWI_OK;
  const unsigned nb = (unsigned)std::min<long long>((n + 255) / 256, 8192);
  axpby_kernel<<<nb, 256, 0, (hipStream_t)stream>>>((long long)n, alpha, x, beta, y, out);
  return hipGetLastError() == hipSuccess ? FWI_OK : FWI_ERR_HIP;
}

fwi_status fwi_absmax(void* stream, int64_t n, const double* x, double* out) {
  if (n < 0 || !out || (n > 0 && !x)) return FWI_ERR_ARG;
  absmax_kernel<<<1, 1024, 0, (hipStream_t)stream>>>((long long)n, x, out);
  return hipGetLastError() == hipSuccess ? FWI_OK : FWI_ERR_HIP;
}

static bool conv_shape(const fwi_conv_shape* s, ConvShape& c) {
  if (!s || s->N < 1 || s->Ci < 1 || s->D < 1 || s->H < 1 || s->W < 1 || s->Co < 1) return false;
  if ((s->K != 1 && s->K != 3) || s->sd < 1 || s->sh < 1 || s->sw < 1) return false;
  c = ConvShape{s->N, s->Ci, s->D, s->H, s->W, s->Co, s->K, s->sd, s->sh, s->sw,
                conv_out(s->D, s->K, s->sd), conv_out(s->H, s->K, s->sh), conv_out(s->W, s->K, s->sw)};
  return c.Do >= 1 && c.Ho >= 1 && c.Wo >= 1;
}

fwi_status fwi_conv3d_forward(void* stream, const fwi_conv_shape* shape, const float* x, const float* w,
                              const float* b, int relu, float* y) {
  ConvShape c;
  if (!conv_shape(shape, c) || !x || !w || !y) return FWI_ERR_ARG;
  const long long n = (long long)c.N * c.Co * c.Do * c.Ho * c.Wo;
  conv3d_forward_kernel<<<(unsigned)((n + 255) / 256), 256, 0, (hipStream_t)stream>>>(c, x, w, b, relu, y);
  return hipGetLastError() == hipSuccess ? FWI_OK : FWI_ERR_HIP;
}

fwi_status fwi_to_bf16(void* stream, int64_t n, const float* in, uint16_t* out) {
  if (n < 0 || (n > 0 && (!in || !out))) return FWI_ERR_ARG;
  if (n == 0) return FWI_OK;
  const unsigned nb = (unsigned)std::min<long long>((n + 255) / 256, 8192);
  to_bf16_kernel<<<nb, 256, 0, (hipStream_t)stream>>>((long long)n, in, (unsigned short*)out);
  return hipGetLastError() == hipSuccess ? FWI_OK : FWI_ERR_HIP;
}

fwi_status fwi_conv3d_forward_bf16(void* stream, const fwi_conv_shape* shape, const uint16_t* x, const uint16_t* w,
                                   const float* b, int relu, int out_fp32, void* y) {
  ConvShape c;
  if (!conv_shape(shape, c) || !x || !w || !y) return FWI_ERR_ARG;
  const long long P = (long long)c.Do * c.Ho * c.Wo;
  if (c.N > 65535) return FWI_ERR_ARG;
  const dim3 grid((unsigned)((P + 63) / 64), (unsigned)c.N);
  conv3d_bf16_mfma_kernel<<<grid, CONV_MFMA_THREADS, 0, (hipStream_t)stream>>>(
      c, (const unsigned short*)x, (const unsigned short*)w, b, relu, out_fp32, y);
  return hipGetLastError() == hipSuccess ? FWI_OK : FWI_ERR_HIP;
}

fwi_status fwi_conv3d_backward(void* stream, const fwi_conv_shape* shape, const float* x, const float* w,
                               const float* y, const float* dy, int relu, float* dx, float* dw, float* db) {
  ConvShape c;
  if (!conv_shape(shape, c) || !x || !w || !dy || (relu && !y) || !dw) return FWI_ERR_ARG;
  hipStream_t st = (hipStream_t)stream;
  if (dx) {
    const long long n = (long long)c.N * c.Ci * c.D * c.H * c.W;
    conv3d_backward_data_kernel<<<(unsigned)((n + 255) / 256), 256, 0, st>>>(c, dy, y, relu, w, dx);
  }
  conv3d_backward_weight_kernel<<<(unsigned)(c.Co * c.Ci * c.K * c.K * c.K), 256, 0, st>>>(c, dy, y, relu, x, dw);
  if (db) conv3d_backward_bias_kernel<<<(unsigned)c.Co, 256, 0, st>>>(c, dy, y, relu, db);
  return hipGetLastError() == hipSuccess ? FWI_OK : FWI_ERR_HIP;
}

fwi_status fwi_mse(void* stream, int64_t n, const float* y, const float* t, float* loss, float* grad) {
  if (n < 1 || !y || !t || (!loss && !grad)) return FWI_ERR_ARG;
  mse_kernel<<<1, 1024, 0, (hipStream_t)stream>>>((long long)n, y, t, loss, grad);
  return hipGetLastError() == hipSuccess ? FWI_OK : FWI_ERR_HIP;
}

fwi_status fwi_adam(void* stream, int64_t n, float* param, const float* grad, float* m, float* v, float lr,
                    float beta1, float beta2, float eps, int step) {
  if (n < 1 || !param || !grad || !m || !v || step < 1) return FWI_ERR_ARG;
  adam_kernel<<<(unsigned)((n + 255) / 256), 256, 0, (hipStream_t)stream>>>((long long)n, param, grad, m, v, lr,
                                                                            beta1, beta2, eps, step);
  return hipGetLastError() == hipSuccess ? FWI_OK : FWI_ERR_HIP;
}

fwi_status fwi_trace_features(void* stream, const double* traces, int nsrc, int nsteps, int nrec,
                              const int32_t* rec_idx, int hw, int T, int t0, int tstride, int comp, float scale,
                              float* out) {
  if (!traces || !rec_idx || !out || nsrc < 1 || nsteps < 1 || nrec < 1 || hw < 1 || T < 1 || t0 < 0 ||
      tstride < 1 || comp < 0 || comp > 2)
    return FWI_ERR_ARG;
  const long long n = (long long)nsrc * T * hw;
  trace_features_kernel<<<(unsigned)((n + 255) / 256), 256, 0, (hipStream_t)stream>>>(
      traces, nsrc, nsteps, nrec, rec_idx, hw, T, t0, tstride, comp, scale, out);
  return hipGetLastError() == hipSuccess ? FWI_OK : FWI_ERR_HIP;
}

fwi_status fwi_grid_to_nodes(fwi_plan* p, void* stream, const float* coarse, int gx, int gy, int gz,
                             const double* base, double* out) {
  if (!p) return FWI_ERR_ARG;
  if (!coarse || !base || !out || gx < 1 || gy < 1 || gz < 1)
    return fail(p, FWI_ERR_ARG, "fwi_grid_to_nodes: bad argument");
  const Geo& G = p->g;
  grid_to_nodes_kernel<<<blocks(G.n_int, 256), 256, 0, (hipStream_t)stream>>>(coarse, gx, gy, gz, G.NIX, G.NIY,
                                                                               G.NIZ, base, out);
  HIP_TRY(p, hipGetLastError());
  return FWI_OK;
}

const char* fwi_status_string(fwi_status s) {
  switch (s) {
    case FWI_OK: return "ok";
    case FWI_ERR_ARG: return "invalid argument";
    case FWI_ERR_SHAPE: return "unsupported mesh or time axis";
    case FWI_ERR_HIP: return "HIP runtime error";
    case FWI_ERR_STATE: return "call order violated";
    case FWI_ERR_UNSTABLE: return "time step above the stability bound";
    case FWI_ERR_NOMEM: return "out of host memory";
  }
  return "unknown status";
}

const char* fwi_last_error(const fwi_plan* p) { return p ? p->err.c_str() : g_plan_err.c_str(); }

}  // extern "C"
