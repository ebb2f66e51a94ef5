// Problem objects, the twogrid V-cycle sequence, the FGMRES(m) driver and the C ABI.
//
// The device holds every vector and operator; the host only runs the O(m^2) work of the
// small Hessenberg least-squares problem (complex Givens rotations, back substitution)
// after one small read-back per iteration, exactly as the outer method prescribes
// (Sec. 4: right-preconditioned flexible GMRES on A_0 with a V-cycle on A_eps).

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <condition_variable>
#include <deque>
#include <limits>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <thread>

#include "hz_internal.h"

namespace hz {

static thread_local std::string g_err;
void set_error(const std::string& msg) { g_err = msg; }

struct OomError {
  size_t bytes;
};

// Owner of the device allocations of one object, with byte accounting.
struct DevMem {
  std::vector<std::pair<void*, size_t>> live;
  size_t bytes = 0;
  template <typename T> T* alloc(size_t n) {
    void* p = nullptr;
    const size_t nb = std::max<size_t>(n, 1) * sizeof(T);
    if (hipMalloc(&p, nb) != hipSuccess) {
      (void)hipGetLastError();
      throw OomError{nb};
    }
    live.emplace_back(p, nb);
    bytes += nb;
    return static_cast<T*>(p);
  }
  void release(void* p) {
    for (size_t i = 0; i < live.size(); ++i)
      if (live[i].first == p) {
        (void)hipFree(p);
        bytes -= live[i].second;
        live.erase(live.begin() + i);
        return;
      }
  }
  // Stream-ordered allocation for buffers that live only during setup: hipFree may wait for
  // the whole device, which would serialise concurrent setups; hipFreeAsync does not.
  template <typename T> T* alloc_async(size_t n, hipStream_t st) {
    void* p = nullptr;
    const size_t nb = std::max<size_t>(n, 1) * sizeof(T);
    if (hipMallocAsync(&p, nb, st) != hipSuccess) {
      (void)hipGetLastError();
      return alloc<T>(n);
    }
    async.emplace_back(p, nb);
    bytes += nb;
    return static_cast<T*>(p);
  }
  void release_async(void* p, hipStream_t st) {
    for (size_t i = 0; i < async.size(); ++i)
      if (async[i].first == p) {
        (void)hipFreeAsync(p, st);
        bytes -= async[i].second;
        async.erase(async.begin() + i);
        return;
      }
    release(p);
  }
  std::vector<std::pair<void*, size_t>> async;
  ~DevMem() {
    for (auto& a : live) (void)hipFree(a.first);
    for (auto& a : async) (void)hipFree(a.first);
  }
};

template <typename T> struct Scratch {
  // V-cycle scratch for up to `cap` right-hand sides: fine vectors with stride N, coarse
  // vectors with stride Nc.
  V2<T>*ua = nullptr, *ub = nullptr, *rf = nullptr, *rc = nullptr, *ec = nullptr;
  V2<T>* ff = nullptr;   // FP32 copy of the V-cycle input (mixed precision)
  int cap = 0;
};

template <typename T> struct Level {
  DevOp<T> fine, coarse;   // A_eps on the fine and coarse lattices
  const T* rw = nullptr;   // prolongation weights
  const V2<T>* S = nullptr;
  CoarseSolveWork cw;
  Scratch<T> sc;
};

// Krylov workspace of a group of solves advancing in lockstep. Every per-solve array has a
// uniform stride; kernels gather their operands through small device offset tables that are
// rebuilt for each step.
struct Workspace {
  int cap = 0, m = 0, prec = HZ_FP64, nblk = 0;
  long N = 0, Nc = 0;
  DevMem mem;
  double2* V = nullptr;     // [cap][m + 1][N] Arnoldi basis
  double2* RW = nullptr;    // [2][cap][N]: residuals r, then Arnoldi vectors w
  double2* Fs = nullptr;    // [cap][N] staged right-hand sides (batched calls)
  double2* Us = nullptr;    // [cap][N] staged solutions (batched calls)
  double2* Zd = nullptr;    // [cap][m][N] preconditioned vectors (FP64)
  float2* Zf = nullptr;     // [cap][m][N] preconditioned vectors (mixed precision)
  double2* partial = nullptr;   // [cap][blocks][64]
  double2* hbuf = nullptr;      // [cap][192]: CGS2 pass 1, pass 2, |w|^2
  double2* red = nullptr;       // [cap][kReduceGroups][64] first-stage sums of the reductions
  char* dreg = nullptr;         // device copies of the two upload regions
  void* gb = nullptr;           // [cap][Nc] coarse forward-sweep buffers (per solve)
  Scratch<double> s64;
  Scratch<float> s32;
  double2* pin = nullptr;       // pinned read-back [cap][192]
  char* up = nullptr;           // pinned upload staging
  size_t up_bytes = 0;
  static constexpr int kTabs = 8;
  ~Workspace() {
    if (pin) (void)hipHostFree(pin);
    if (up) (void)hipHostFree(up);
  }
  double2* r(int q) const { return RW + size_t(q) * N; }
  double2* w(int q) const { return RW + size_t(cap + q) * N; }
};

}  // namespace hz

using namespace hz;

struct hz_problem {
  double k = 0;              // wavenumber (the largest cell value for per-cell k)
  int n = 0, p = 1;
  cd s;
  int cells = 0;             // per-cell k and shift: operators stored per lattice point
  hz_options opt{};
  int M = 0, Mc = 0;
  long N = 0, Nc = 0;
  long G = 0;                 // coarse-solve work per right-hand side (elements)
  CoarseLayout L;
  const MfSym* sym = nullptr; // multifrontal coarse factor (else the block-tridiagonal one)
  MfView* dmf = nullptr;      // device copy of its symbolic data (and hmf, the same view
  MfView hmf;                 // held on the host: device pointers for host-side launches)
  size_t fel = 0;             // coarse factor elements
  DevMem mem;
  // FP64 operators and tables
  double2 *cA0 = nullptr, *cAe = nullptr, *wdAe = nullptr, *cAc = nullptr;
  double* rw = nullptr;
  double2* S = nullptr;
  // FP32 operators and tables
  float2 *fcAe = nullptr, *fwdAe = nullptr, *fcAc = nullptr;
  float* frw = nullptr;
  float2* Sf = nullptr;
  int m = 0;                  // restart capacity
  Scratch<double> s64;        // V-cycle scratch for one right-hand side
  Scratch<float> s32;
  float2 *ax32 = nullptr, *af32 = nullptr, *ay32 = nullptr, *cx32 = nullptr, *cy32 = nullptr;
  std::unique_ptr<Workspace> ws1;   // Krylov workspace of hz_solve (allocated at first use)
  CoarseSolveWork cw;         // forward-sweep buffers and error flag of the coarse solve
  double gl_t[10], gl_w[10], lag[40];
  // quadrature of the point-source load vector: xi, eta, w [nq] each, phi [nloc][nq]; loc
  double* qtab = nullptr;
  int* qloc = nullptr;
  int nq = 0;
  double setup_s = 0;
  std::atomic<int> busy{0};
  // device-time counters (timing mode): event pairs around each coarse-solve launch
  bool timing = false;
  hz_stats stats{};
  std::vector<std::pair<hipEvent_t, hipEvent_t>> ev_free, ev_pending;
  ~hz_problem() {
    ws1.reset();
    for (auto& e : ev_free) { (void)hipEventDestroy(e.first); (void)hipEventDestroy(e.second); }
    for (auto& e : ev_pending) { (void)hipEventDestroy(e.first); (void)hipEventDestroy(e.second); }
  }
};

namespace {

using clk = std::chrono::steady_clock;
double secs(clk::time_point a) { return std::chrono::duration<double>(clk::now() - a).count(); }

hz_status fail(hz_status st, const std::string& msg) {
  set_error(msg);
  return st;
}

hz_status map_exception() {
  try {
    throw;
  } catch (const HipError& e) {
    set_error(std::string("HIP error ") + hipGetErrorString(e.e) + " in " + e.where);
    return e.e == hipErrorOutOfMemory ? HZ_ENOMEM : HZ_EDEVICE;
  } catch (const OomError& e) {
    set_error("device allocation of " + std::to_string(e.bytes) + " bytes failed");
    return HZ_ENOMEM;
  } catch (const std::bad_alloc&) {
    set_error("host allocation failed");
    return HZ_ENOMEM;
  } catch (const std::exception& e) {
    set_error(e.what());
    return HZ_EDEVICE;
  }
}

struct BusyGuard {
  std::atomic<int>& f;
  bool ok;
  explicit BusyGuard(std::atomic<int>& x) : f(x), ok(x.exchange(1) == 0) {}
  ~BusyGuard() {
    if (ok) f.store(0);
  }
};

bool valid_options(const hz_options& o, std::string& why) {
  if (o.nu < 0 || o.nu > 16) { why = "nu must be in [0, 16]"; return false; }
  if (!(o.omega > 0 && o.omega < 2)) { why = "omega must be in (0, 2)"; return false; }
  if (o.restart < 1 || o.restart > 64) { why = "restart must be in [1, 64]"; return false; }
  if (o.maxit < 1) { why = "maxit must be >= 1"; return false; }
  if (!(o.tol >= 0) || !std::isfinite(o.tol)) { why = "tol must be finite and >= 0"; return false; }
  if (o.prec != HZ_FP64 && o.prec != HZ_MIXED) { why = "prec must be HZ_FP64 or HZ_MIXED"; return false; }
  return true;
}

bool valid_problem(double k, double h, int p, cd s, int& n, std::string& why) {
  if (!(k > 0) || !std::isfinite(k)) { why = "k must be finite and > 0"; return false; }
  if (!(h > 0) || !std::isfinite(h)) { why = "h must be finite and > 0"; return false; }
  const double nn = 1.0 / h;
  n = int(std::lround(nn));
  if (std::fabs(nn - n) > 1e-9 * nn || n < 2 || n > 4096 || n % 2) {
    why = "1/h must be an even integer in [2, 4096]";
    return false;
  }
  if (p < 1 || p > 3) { why = "p must be 1, 2 or 3"; return false; }
  if (!std::isfinite(s.real()) || !std::isfinite(s.imag()) || !(s.imag() > 0)) {
    why = "shift multiplier must be finite with Im(s) > 0";
    return false;
  }
  return true;
}

// Gauss-Legendre rule with 10 points on [0, 1] (Newton on the Legendre recurrence).
void gauss_legendre10(double* t, double* w) {
  const int n = 10;
  for (int i = 0; i < n; ++i) {
    double x = std::cos(M_PI * (i + 0.75) / (n + 0.5));
    double dp = 0;
    for (int it = 0; it < 100; ++it) {
      double p0 = 1, p1 = x;
      for (int kk = 2; kk <= n; ++kk) {
        const double p2 = ((2 * kk - 1) * x * p1 - (kk - 1) * p0) / kk;
        p0 = p1;
        p1 = p2;
      }
      dp = n * (x * p1 - p0) / (x * x - 1);
      const double dx = p1 / dp;
      x -= dx;
      if (std::fabs(dx) < 1e-16) break;
    }
    t[i] = 0.5 * (x + 1);
    w[i] = 1.0 / ((1 - x * x) * dp * dp);   // (2 / ((1-x^2) P'^2)) / 2
  }
}

// Coarse direct solver: the multifrontal factor (nested dissection) unless HZ_COARSE=band
// selects the block-tridiagonal factor with the persistent block solve.
bool use_mf() {
  static const bool on = [] {
    const char* e = std::getenv("HZ_COARSE");
    return !(e && std::string(e) == "band");
  }();
  return on;
}

// Bytes of the device copy of a symbolic factor (nodes, point lists, maps, tasks, view).
size_t mf_sym_bytes(const MfSym& y) {
  return y.nodes.size() * sizeof(MfNode) +
         (y.I.size() + y.B.size() + y.map.size() + y.hn.size() + y.inv.size() +
          y.sub_lev.size() + y.sub_bloc.size()) * 4 + y.sub_hdr.size() * sizeof(MfSubHdr) +
         y.sub_node.size() * sizeof(MfSubNode) +
         (y.fwd.size() + y.bwd.size()) * sizeof(MfTask) + sizeof(MfView) + 12 * 256;
}

struct Sizes {
  long N, Nc;
  long G;                  // coarse-solve work per right-hand side (elements)
  size_t factor_elems, maxblock, sym_bytes;
  int nblk;
};
Sizes sizes_of(int n, int p) {
  Sizes z;
  const int M = p * n + 1, Mc = p * (n / 2) + 1;
  z.N = long(M) * M;
  z.Nc = long(Mc) * Mc;
  CoarseLayout L{p, n / 2, Mc};
  z.maxblock = size_t(L.size(0));
  if (use_mf()) {
    const MfSym& y = mf_symbolic(p, n / 2);
    z.factor_elems = size_t(y.numel);
    z.G = std::max(z.Nc, y.uel);
    z.sym_bytes = mf_sym_bytes(y);
  } else {
    z.factor_elems = L.total();
    z.G = z.Nc;
    z.sym_bytes = 0;
  }
  z.nblk = mdot_blocks(z.N);
  return z;
}

// Bytes of the V-cycle scratch for `cap` right-hand sides (G: coarse-solve work each).
size_t scratch_bytes(long N, long Nc, long G, int cap, int prec) {
  const size_t it = prec == HZ_MIXED ? 8 : 16;
  return size_t(cap) * ((prec == HZ_MIXED ? 4 : 3) * size_t(N) + 2 * size_t(Nc)) * it +
         size_t(cap) * G * 16;   // coarse-solve work
}

// Bytes of a Krylov workspace for `cap` solves with restart capacity m (staged: with room
// for copies of the right-hand sides and solutions).
size_t workspace_bytes(long N, int nblk, int cap, int m, int prec, bool staged) {
  size_t b = 0;
  b += size_t(cap) * (m + 1) * N * 16;                          // V
  b += size_t(cap) * m * N * (prec == HZ_MIXED ? 8 : 16);       // Z
  b += 2 * size_t(cap) * N * 16;                                // r, w
  if (staged) b += 2 * size_t(cap) * N * 16;                    // F, u
  b += size_t(cap) * (size_t(fused_blocks(N)) * 64 * 16 + size_t(kReduceGroups) * 64 * 16 +
                      192 * 16 + 64 * 16 + 8);
  b += 2 * size_t(cap) * (Workspace::kTabs * 8 + 2 * 4 + 8 + 3 * 8 + 64 * 16) + 4096;
  return b;
}

// Device bytes a problem holds after its first solve: factor, tables, scratch, workspace.
size_t resident_bytes(int n, int p, int m, int prec) {
  const Sizes z = sizes_of(n, p);
  size_t b = z.factor_elems * (prec == HZ_MIXED ? 8 : 16);
  b += scratch_bytes(z.N, z.Nc, z.G, 1, prec);
  b += workspace_bytes(z.N, z.nblk, 1, m, prec, false);
  b += 64 * 1024 + 4 * size_t(z.G) * 16 + 256 + z.sym_bytes;   // tables, coarse-solve buffers
  return b;
}

void upload_tables(hz_problem* pr, hipStream_t st) {
  const LevelTables ft = build_level_tables(pr->p, pr->n, 1.0 / pr->n);
  const LevelTables ct = build_level_tables(pr->p, pr->n / 2, 2.0 / pr->n);
  const std::vector<cd> a0 = combine_operator(ft, pr->k, cd(1.0, 0.0));
  const std::vector<cd> ae = combine_operator(ft, pr->k, pr->s);
  const std::vector<cd> ac = combine_operator(ct, pr->k, pr->s);
  const int p = pr->p, W2 = (2 * p + 1) * (2 * p + 1), nreg = p * p * 9;
  std::vector<cd> wd(nreg, cd(0, 0));
  for (int i = 0; i < nreg; ++i) {
    const cd d = ae[size_t(i) * W2 + (W2 - 1) / 2];
    if (std::abs(d) > 0) wd[i] = pr->opt.omega / d;
  }
  auto up2 = [&](const std::vector<cd>& v, double2*& d, float2*& f, bool want_f) {
    d = pr->mem.alloc<double2>(v.size());
    HZ_HIP(hipMemcpyAsync(d, v.data(), v.size() * 16, hipMemcpyHostToDevice, st));
    if (want_f) {
      std::vector<float2> fv(v.size());
      for (size_t i = 0; i < v.size(); ++i) fv[i] = make_float2(float(v[i].real()), float(v[i].imag()));
      f = pr->mem.alloc<float2>(v.size());
      HZ_HIP(hipMemcpyAsync(f, fv.data(), v.size() * 8, hipMemcpyHostToDevice, st));
      HZ_HIP(hipStreamSynchronize(st));   // fv is local
    }
  };
  float2* dummy = nullptr;
  up2(a0, pr->cA0, dummy, false);
  up2(ae, pr->cAe, pr->fcAe, true);
  up2(wd, pr->wdAe, pr->fwdAe, true);
  up2(ac, pr->cAc, pr->fcAc, true);
  pr->rw = pr->mem.alloc<double>(ft.RW.size());
  HZ_HIP(hipMemcpyAsync(pr->rw, ft.RW.data(), ft.RW.size() * 8, hipMemcpyHostToDevice, st));
  std::vector<float> frw(ft.RW.begin(), ft.RW.end());
  pr->frw = pr->mem.alloc<float>(frw.size());
  HZ_HIP(hipMemcpyAsync(pr->frw, frw.data(), frw.size() * 4, hipMemcpyHostToDevice, st));
  {
    const QuadTables qt = build_quad_tables(p, 6);
    pr->nq = qt.nq;
    std::vector<double> q;
    q.insert(q.end(), qt.xi.begin(), qt.xi.end());
    q.insert(q.end(), qt.eta.begin(), qt.eta.end());
    q.insert(q.end(), qt.w.begin(), qt.w.end());
    q.insert(q.end(), qt.phi.begin(), qt.phi.end());
    pr->qtab = pr->mem.alloc<double>(q.size());
    HZ_HIP(hipMemcpyAsync(pr->qtab, q.data(), q.size() * 8, hipMemcpyHostToDevice, st));
    pr->qloc = pr->mem.alloc<int>(qt.loc.size());
    HZ_HIP(hipMemcpyAsync(pr->qloc, qt.loc.data(), qt.loc.size() * 4, hipMemcpyHostToDevice, st));
    HZ_HIP(hipStreamSynchronize(st));
  }
  HZ_HIP(hipStreamSynchronize(st));   // the host tables are local
  gauss_legendre10(pr->gl_t, pr->gl_w);
  for (int l = 0; l < 4; ++l)
    for (int q = 0; q < 10; ++q) {
      double v = 1.0;
      for (int mm = 0; mm <= p; ++mm)
        if (mm != l) v *= (pr->gl_t[q] - double(mm) / p) / (double(l) / p - double(mm) / p);
      pr->lag[l * 10 + q] = (l <= p) ? v : 0.0;
    }
}

// Per-point operators of a problem with per-cell k and shift (row-major [j][i] host arrays of
// the n x n fine cells): A_0 (s = 1) and A_s with the Jacobi multipliers on the fine lattice,
// A_s on the coarse lattice (the Galerkin operator), all assembled on the device, plus their
// FP32 copies. Replaces the class-table operators of upload_tables.
void upload_cells(hz_problem* pr, const double* k_cell, const hz_c64* s_cell, hipStream_t st) {
  const int p = pr->p, n = pr->n, W2 = (2 * p + 1) * (2 * p + 1);
  const long nc2 = long(n) * n;
  const CellTables ft = build_cell_tables(p, 1, 1.0 / n);
  const CellTables ct = build_cell_tables(p, 2, 1.0 / n);
  std::vector<double2> sv(nc2);
  for (long c = 0; c < nc2; ++c) sv[c] = make_double2(s_cell[c].re, s_cell[c].im);
  auto up = [&](const void* h, size_t bytes) {
    void* d = pr->mem.alloc_async<char>(bytes, st);
    HZ_HIP(hipMemcpyAsync(d, h, bytes, hipMemcpyHostToDevice, st));
    return d;
  };
  std::vector<void*> tmp;
  auto upd = [&](const std::vector<double>& v) {
    tmp.push_back(up(v.data(), v.size() * 8));
    return static_cast<const double*>(tmp.back());
  };
  const double *fK = upd(ft.K), *fM = upd(ft.Mm), *fB = upd(ft.B);
  const double *cK = upd(ct.K), *cM = upd(ct.Mm), *cB = upd(ct.B);
  tmp.push_back(up(k_cell, nc2 * 8));
  const double* dk = static_cast<const double*>(tmp.back());
  tmp.push_back(up(sv.data(), nc2 * 16));
  const double2* ds = static_cast<const double2*>(tmp.back());
  pr->cA0 = pr->mem.alloc<double2>(size_t(W2) * pr->N);
  pr->cAe = pr->mem.alloc<double2>(size_t(W2) * pr->N);
  pr->wdAe = pr->mem.alloc<double2>(pr->N);
  pr->cAc = pr->mem.alloc<double2>(size_t(W2) * pr->Nc);
  launch_assemble_cells(p, 1, pr->M, fK, fM, fB, dk, nullptr, pr->opt.omega, pr->cA0, nullptr, st);
  launch_assemble_cells(p, 1, pr->M, fK, fM, fB, dk, ds, pr->opt.omega, pr->cAe, pr->wdAe, st);
  launch_assemble_cells(p, 2, pr->Mc, cK, cM, cB, dk, ds, pr->opt.omega, pr->cAc, nullptr, st);
  pr->fcAe = pr->mem.alloc<float2>(size_t(W2) * pr->N);
  pr->fwdAe = pr->mem.alloc<float2>(pr->N);
  pr->fcAc = pr->mem.alloc<float2>(size_t(W2) * pr->Nc);
  launch_d2f(pr->cAe, pr->fcAe, long(W2) * pr->N, st);
  launch_d2f(pr->wdAe, pr->fwdAe, pr->N, st);
  launch_d2f(pr->cAc, pr->fcAc, long(W2) * pr->Nc, st);
  HZ_HIP(hipStreamSynchronize(st));   // the host arrays are the caller's / local
  for (void* d : tmp) pr->mem.release_async(d, st);
}

// The problem's view of its mesh class's symbolic multifrontal data (shared, per device).
void upload_symbolic(hz_problem* pr, hipStream_t st) {
  pr->dmf = mf_device_view(*pr->sym, &pr->hmf, st);
}


template <typename T>
void alloc_scratch(DevMem& mem, Scratch<T>& sc, int cap, long N, long Nc, bool with_ff) {
  sc.cap = cap;
  sc.ua = mem.alloc<V2<T>>(size_t(cap) * N);
  sc.ub = mem.alloc<V2<T>>(size_t(cap) * N);
  sc.rf = mem.alloc<V2<T>>(size_t(cap) * N);
  if (with_ff) sc.ff = mem.alloc<V2<T>>(size_t(cap) * N);
  sc.rc = mem.alloc<V2<T>>(size_t(cap) * Nc);
  sc.ec = mem.alloc<V2<T>>(size_t(cap) * Nc);
}

void ensure_fp64_work(hz_problem* pr) {
  if (pr->s64.cap) return;
  alloc_scratch<double>(pr->mem, pr->s64, 1, pr->N, pr->Nc, false);
}

void ensure_mixed_work(hz_problem* pr, hipStream_t st) {
  if (!pr->Sf) {
    pr->Sf = pr->mem.alloc<float2>(pr->fel);
    launch_factor_to_f32(pr->S, pr->Sf, pr->fel, st);
  }
  if (pr->s32.cap) return;
  alloc_scratch<float>(pr->mem, pr->s32, 1, pr->N, pr->Nc, true);
}

void ensure_apply32(hz_problem* pr) {
  if (pr->ax32) return;
  pr->ax32 = pr->mem.alloc<float2>(pr->N);
  pr->af32 = pr->mem.alloc<float2>(pr->N);
  pr->ay32 = pr->mem.alloc<float2>(pr->N);
  pr->cx32 = pr->mem.alloc<float2>(pr->Nc);
  pr->cy32 = pr->mem.alloc<float2>(pr->Nc);
}

// Upload staging of one phase: offset tables, counts, scale factors, Hessenberg solutions.
struct Region {
  long* tab;        // [kTabs][cap] element offsets
  int* itab;        // [2][cap] counts
  double* scl;      // [cap] scale factors
  const void** ptab;  // [kPtrTabs][cap] per-element operator tables
  double2* y;       // [cap][64] Hessenberg solutions
};
constexpr int kPtrTabs = 3;
size_t region_bytes(int cap) {
  auto al = [](size_t b) { return (b + 15) / 16 * 16; };
  return al(size_t(Workspace::kTabs) * cap * 8) + al(size_t(2) * cap * 4) + al(size_t(cap) * 8) +
         al(size_t(kPtrTabs) * cap * 8) + size_t(cap) * 64 * 16;
}
Region region_at(char* base, int cap) {
  auto al = [](size_t b) { return (b + 15) / 16 * 16; };
  Region r;
  size_t o = 0;
  r.tab = reinterpret_cast<long*>(base + o);
  o += al(size_t(Workspace::kTabs) * cap * 8);
  r.itab = reinterpret_cast<int*>(base + o);
  o += al(size_t(2) * cap * 4);
  r.scl = reinterpret_cast<double*>(base + o);
  o += al(size_t(cap) * 8);
  r.ptab = reinterpret_cast<const void**>(base + o);
  o += al(size_t(kPtrTabs) * cap * 8);
  r.y = reinterpret_cast<double2*>(base + o);
  return r;
}

std::unique_ptr<Workspace> make_workspace(int cap, int m, int prec, long N, long Nc, long G,
                                          int rcap, bool staged) {
  std::unique_ptr<Workspace> w(new Workspace());
  w->cap = cap; w->m = m; w->prec = prec; w->N = N; w->Nc = Nc; w->nblk = mdot_blocks(N);
  w->V = w->mem.alloc<double2>(size_t(cap) * (m + 1) * N);
  w->RW = w->mem.alloc<double2>(2 * size_t(cap) * N);
  if (staged) {
    w->Fs = w->mem.alloc<double2>(size_t(cap) * N);
    w->Us = w->mem.alloc<double2>(size_t(cap) * N);
  }
  if (prec == HZ_MIXED) w->Zf = w->mem.alloc<float2>(size_t(cap) * m * N);
  else w->Zd = w->mem.alloc<double2>(size_t(cap) * m * N);
  w->partial = w->mem.alloc<double2>(size_t(cap) * fused_blocks(N) * 64);
  w->hbuf = w->mem.alloc<double2>(size_t(cap) * 192);
  w->red = w->mem.alloc<double2>(size_t(cap) * kReduceGroups * 64);
  w->up_bytes = region_bytes(cap);
  // device mirror of the two upload regions
  w->dreg = w->mem.alloc<char>(2 * w->up_bytes);
  if (rcap > 0) {
    if (prec == HZ_MIXED) alloc_scratch<float>(w->mem, w->s32, rcap, N, Nc, true);
    else alloc_scratch<double>(w->mem, w->s64, rcap, N, Nc, false);
    w->gb = w->mem.alloc<double2>(size_t(rcap) * G);
  }
  HZ_HIP(hipHostMalloc(reinterpret_cast<void**>(&w->pin), size_t(cap) * 192 * 16, hipHostMallocDefault));
  HZ_HIP(hipHostMalloc(reinterpret_cast<void**>(&w->up), 2 * w->up_bytes, hipHostMallocDefault));
  return w;
}

Level<double> level64(hz_problem* pr, const Scratch<double>& sc) {
  Level<double> l;
  l.fine = DevOp<double>{pr->cAe, pr->wdAe, pr->M};
  l.coarse = DevOp<double>{pr->cAc, nullptr, pr->Mc};
  l.fine.pn = l.coarse.pn = pr->cells;
  l.rw = pr->rw;
  l.S = pr->S;
  l.cw = pr->cw;
  l.sc = sc;
  return l;
}
Level<float> level32(hz_problem* pr, const Scratch<float>& sc) {
  Level<float> l;
  l.fine = DevOp<float>{pr->fcAe, pr->fwdAe, pr->M};
  l.coarse = DevOp<float>{pr->fcAc, nullptr, pr->Mc};
  l.fine.pn = l.coarse.pn = pr->cells;
  l.rw = pr->frw;
  l.S = pr->Sf;
  l.cw = pr->cw;
  l.sc = sc;
  return l;
}

// Timing mode: event pairs around the coarse-solve launches, summed when complete.
std::pair<hipEvent_t, hipEvent_t> take_events(hz_problem* pr) {
  if (pr->ev_free.empty()) {
    hipEvent_t a, b;
    HZ_HIP(hipEventCreate(&a));
    HZ_HIP(hipEventCreate(&b));
    pr->ev_free.emplace_back(a, b);
  }
  auto e = pr->ev_free.back();
  pr->ev_free.pop_back();
  return e;
}
void collect_timing(hz_problem* pr, bool wait) {
  std::vector<std::pair<hipEvent_t, hipEvent_t>> keep;
  for (auto& e : pr->ev_pending) {
    if (!wait && hipEventQuery(e.second) != hipSuccess) {
      (void)hipGetLastError();
      keep.push_back(e);
      continue;
    }
    HZ_HIP(hipEventSynchronize(e.second));
    float ms = 0;
    HZ_HIP(hipEventElapsedTime(&ms, e.first, e.second));
    pr->stats.coarse_solve_ms += ms;
    pr->ev_free.push_back(e);
  }
  pr->ev_pending.swap(keep);
}

// Algorithmic bytes of one coarse solve job: the stored factor read twice (the last block
// once) plus, per right-hand side, the coarse vector read and the solution written and
// re-read.
// Multifrontal solve: every stored matrix read once (S and G^T forward, G backward), plus per
// right-hand side the coarse vector read, the solution written and re-read.
double mf_job_bytes(const MfSym& y, size_t item, int nrhs) {
  const double mc2 = double(y.Mc) * y.Mc;
  return double(y.numel) * item + 3.0 * mc2 * item * nrhs;
}

// Block-tridiagonal factor: per block j the Schur complement products and the inverse of the
// (p Mc)^2 block, about 3 (p Mc)^3 complex multiply-adds.
double band_factor_flop(const CoarseLayout& L) {
  const double b = double(L.p) * L.Mc;
  return 8.0 * 3.0 * b * b * b * L.nc;
}

double csolve_job_bytes(const CoarseLayout& L, size_t item, int nrhs) {
  const double mc2 = double(L.Mc) * L.Mc;
  return (2.0 * double(L.total()) - mc2) * item + 3.0 * mc2 * item * nrhs;
}

// Coarse solves of jobs (timed with HIP events on the stream when the first problem was
// created with timing; counters accumulate in that problem).
template <typename T>
void timed_coarse_jobs(hz_problem* pr, const CoarseJob<T>* jobs, int njobs, hipStream_t st,
                       const CoarseSolveWork* cw = nullptr) {
  double bytes = 0;
  for (int i = 0; i < njobs; ++i)
    bytes += pr->sym ? mf_job_bytes(*pr->sym, sizeof(V2<T>), jobs[i].nrhs)
                     : csolve_job_bytes(pr->L, sizeof(V2<T>), jobs[i].nrhs);
  // a caller-given work set (the allocation-free apply) is never timed: no events are made
  const bool timed = pr->timing && !cw;
  if (!cw) cw = &pr->cw;
  std::pair<hipEvent_t, hipEvent_t> e{};
  if (timed) {
    e = take_events(pr);
    HZ_HIP(hipEventRecord(e.first, st));
  }
  if (pr->sym)
    pr->stats.coarse_solves += mf_solve_jobs<T>(*pr->sym, jobs, njobs, pr->Nc, st);
  else
    pr->stats.coarse_solves += coarse_solve_jobs<T>(pr->L, jobs, njobs, pr->Nc, cw->err,
                                                    cw->persistent, st);
  pr->stats.coarse_bytes += bytes;
  for (int i = 0; i < njobs; ++i) pr->stats.coarse_systems += jobs[i].nrhs;
  if (timed) {
    HZ_HIP(hipEventRecord(e.second, st));
    pr->ev_pending.push_back(e);
    if (pr->ev_pending.size() > 64) collect_timing(pr, true);
  }
}

template <typename T> const V2<T>* factor_of(const hz_problem* pr);
template <> const double2* factor_of<double>(const hz_problem* pr) { return pr->S; }
template <> const float2* factor_of<float>(const hz_problem* pr) { return pr->Sf; }
template <typename T> const V2<T>* coarse_coef_of(const hz_problem* pr);
template <> const double2* coarse_coef_of<double>(const hz_problem* pr) { return pr->cAc; }
template <> const float2* coarse_coef_of<float>(const hz_problem* pr) { return pr->fcAc; }

// One twogrid V(nu, nu)-cycle from a zero initial guess (Algorithm 1, two levels) for nb
// solves of one mesh class at once: nu damped Jacobi sweeps, r_c = P^T (f - A_eps u),
// e_c = A_c^{-1} r_c, u += P e_c, nu sweeps. Solve b uses problem probs[zp[b]] (consecutive
// solves of one problem form one coarse job of up to 4 right-hand sides), input f + af.at(b),
// output z + az.at(b); fine gives the per-solve operators. The iterates live in scratch
// (stride N, coarse stride Nc); gb holds nb coarse forward-sweep buffers (stride Nc).
enum VcPhase { VC_PRE = 1, VC_COARSE = 2, VC_POST = 4, VC_ALL = 7 };

template <typename T>
void vcycle_group(hz_problem* const* probs, const int* zp, int nb, const DevOp<T>& fine,
                  const T* rw, const Scratch<T>& sc, V2<T>* gb, const V2<T>* f, Addr af,
                  V2<T>* z, Addr az, hipStream_t st, int phases = VC_ALL,
                  const CoarseSolveWork* cw = nullptr) {
  hz_problem* pr0 = probs[zp[0]];
  const int p = pr0->p, nu = pr0->opt.nu;
  const long N = pr0->N, Nc = pr0->Nc;
  if (nb > sc.cap) throw std::runtime_error("V-cycle batch exceeds its scratch");
  // buffers: jacobi0 writes ua, each further sweep alternates, so after nu - 1 sweeps the
  // iterate is in ua (nu odd) or ub (nu even)
  V2<T>* cur = (nu % 2 == 1) ? sc.ua : sc.ub;
  V2<T>* nxt = (nu % 2 == 1) ? sc.ub : sc.ua;
  if (phases & VC_PRE) {
    if (nu == 0) {
      // u = 0: the cycle is the coarse correction alone, z = P A_c^{-1} P^T f
      launch_restrict<T>(p, pr0->M, pr0->Mc, rw, f, sc.rc, nb, af, Addr(Nc), st);
    } else {
      // sweep s leaves the iterate in ua (s odd) or ub (s even); the first two sweeps from
      // zero run as one pass
      V2<T>* c = sc.ua;
      V2<T>* x = sc.ub;
      if (nu == 1) {
        launch_jacobi0<T, T>(p, fine, f, af, c, Addr(N), nb, st);
      } else {
        launch_stencil<T, T, T, T>(p, ST_SMOOTH0, fine, f, af, f, af, x, Addr(N), nb, st);
        std::swap(c, x);
      }
      for (int sw = 2; sw < nu; ++sw) {
        launch_stencil<T, T, T, T>(p, ST_SMOOTH, fine, c, Addr(N), f, af, x, Addr(N), nb, st);
        std::swap(c, x);
      }
      if (!launch_resid_restrict<T>(p, fine, c, Addr(N), f, af, pr0->Mc, rw, sc.rc, Addr(Nc), nb,
                                    st)) {
        launch_stencil<T, T, T, T>(p, ST_RESID, fine, c, Addr(N), f, af, sc.rf, Addr(N), nb, st);
        launch_restrict<T>(p, pr0->M, pr0->Mc, rw, sc.rf, sc.rc, nb, Addr(N), Addr(Nc), st);
      }
    }
  }
  if (phases & VC_COARSE) {
    // coarse jobs: runs of solves of one problem, at most the LDS group size per job
    const int grp = coarse_group<T>(pr0->L);
    std::vector<CoarseJob<T>> jobs;
    for (int b0 = 0; b0 < nb;) {
      int b1 = b0;
      while (b1 < nb && zp[b1] == zp[b0] && b1 - b0 < grp) ++b1;
      hz_problem* pi = probs[zp[b0]];
      pi->stats.vcycles += b1 - b0;
      CoarseJob<T> j;
      j.S = factor_of<T>(pi);
      j.coef = coarse_coef_of<T>(pi);
      j.pn = pi->cells;
      j.mf = pi->dmf;
      j.ustride = pr0->G;
      j.b = sc.rc + b0 * Nc;
      j.y = sc.ec + b0 * Nc;
      j.gbuf = gb + b0 * pr0->G;
      j.nrhs = b1 - b0;
      jobs.push_back(j);
      b0 = b1;
    }
    timed_coarse_jobs<T>(pr0, jobs.data(), int(jobs.size()), st, cw);
  }
  if (phases & VC_POST) {
    if (nu == 0) {
      launch_prolong<T>(p, pr0->M, pr0->Mc, rw, sc.ec, z, false, nb, az, Addr(Nc), st);
      return;
    }
    // the first post-sweep stages u + P e_c itself where the kernel provides it
    int sw0 = 0;
    if (launch_smooth_pc<T>(p, fine, cur, Addr(N), sc.ec, Addr(Nc), pr0->Mc, rw, f, af,
                            nu == 1 ? z : nxt, nu == 1 ? az : Addr(N), nb, st)) {
      if (nu == 1) return;
      std::swap(cur, nxt);
      sw0 = 1;
    } else {
      launch_prolong<T>(p, pr0->M, pr0->Mc, rw, sc.ec, cur, true, nb, Addr(N), Addr(Nc), st);
    }
    for (int sw = sw0; sw < nu; ++sw) {
      if (sw == nu - 1) {
        launch_stencil<T, T, T, T>(p, ST_SMOOTH, fine, cur, Addr(N), f, af, z, az, nb, st);
      } else {
        launch_stencil<T, T, T, T>(p, ST_SMOOTH, fine, cur, Addr(N), f, af, nxt, Addr(N), nb, st);
        std::swap(cur, nxt);
      }
    }
  }
}

// Single-problem forms used by hz_apply: one right-hand side, the coarse-solve work of the
// level (the problem's own, or the caller's for the allocation-free apply).
template <typename T>
void vcycle(hz_problem* pr, const Level<T>& lv, const V2<T>* f, V2<T>* z, hipStream_t st,
            bool own_work) {
  hz_problem* const probs[1] = {pr};
  const int zp[1] = {0};
  vcycle_group<T>(probs, zp, 1, lv.fine, lv.rw, lv.sc, reinterpret_cast<V2<T>*>(lv.cw.g), f,
                  Addr(), z, Addr(), st, VC_ALL, own_work ? nullptr : &lv.cw);
}
template <typename T>
void timed_coarse_solve(hz_problem* pr, const Level<T>& lv, const V2<T>* b, V2<T>* y,
                        hipStream_t st, bool own_work) {
  CoarseJob<T> j;
  j.S = lv.S;
  j.coef = lv.coarse.coef;
  j.pn = lv.coarse.pn;
  j.mf = pr->dmf;
  j.ustride = pr->G;
  j.b = b;
  j.y = y;
  j.gbuf = reinterpret_cast<V2<T>*>(lv.cw.g);
  j.nrhs = 1;
  timed_coarse_jobs<T>(pr, &j, 1, st, own_work ? nullptr : &lv.cw);
}

// Complex Givens rotation with c real: [c s; -conj(s) c] [a; b] = [r; 0].
void givens(cd a, cd b, double& c, cd& s) {
  if (a == cd(0, 0)) {
    c = 0;
    s = cd(1, 0);
    return;
  }
  const double r = std::sqrt(std::norm(a) + std::norm(b));
  c = std::abs(a) / r;
  s = (a / std::abs(a)) * std::conj(b) / r;
}

// Host state of one FGMRES(m) solve (Sec. 4, after Saad 1993).
struct SolveState {
  int prob = 0;
  double normF = 0, beta = 0, est = 1, true_rel = 1, scale = 0;
  int its = 0, j = 0;
  bool restart = true;        // next step starts a cycle: v_0 = r / beta (else v_j = w / h)
  bool done = false, conv = false, ending = false;
  std::vector<cd> H, g;
  std::vector<double> cs;
  std::vector<cd> sn;
  double* hist = nullptr;
  int m = 0;
  clk::time_point t0;
  cd& Hat(int i, int jj) { return H[size_t(i) * m + jj]; }
};

// nsol = nprob * nrhs FGMRES(o.restart) solves advancing in lockstep: every round performs
// one Arnoldi step of each unfinished solve, with the fine kernels and the Arnoldi kernels
// launched once for all of them and the V-cycles of one problem's right-hand sides sharing
// each read of its coarse factor. Solve q belongs to problem q / nrhs; its right-hand side
// and solution are at Fb + foff[q] and Ub + uoff[q]. Each solve follows exactly the steps
// (and floating-point order) it would follow alone. The phases are separate so that a
// caller can interleave the rounds of several groups on one stream:
//   start()   norms of F, u = 0, r = F                                  (synchronises)
//   issue()   queue one round: v_j, V-cycles, A_0 z_j, CGS2, read-back   (asynchronous)
//   complete() after the stream is synchronised: Hessenberg column, rotations, estimate;
//             cycle ends (u += Z y, true residual)                      (synchronises)
struct Lockstep {
  hz_problem* const* probs = nullptr;
  int nprob = 0, nrhs = 0, nsol = 0;
  const double2* Fb = nullptr;
  const long* foff = nullptr;
  double2* Ub = nullptr;
  const long* uoff = nullptr;
  Workspace* ws = nullptr;
  hz_options o{};
  std::vector<SolveState> S;
  std::vector<int> act, end, zp;
  std::vector<cd> y;
  clk::time_point t0;
  bool issued = false;
  int round_nv = 64;        // largest basis size of the round's projections

  ~Lockstep() {
    drop_graphs();
    if (cap_st) (void)hipStreamDestroy(cap_st);
  }
  Lockstep(const Lockstep&) = delete;
  Lockstep& operator=(const Lockstep&) = delete;
  Lockstep(hz_problem* const* probs_, int nprob_, int nrhs_, const double2* Fb_,
           const long* foff_, double2* Ub_, const long* uoff_, Workspace& ws_,
           const hz_options& o_)
      : probs(probs_), nprob(nprob_), nrhs(nrhs_), nsol(nprob_ * nrhs_), Fb(Fb_), foff(foff_),
        Ub(Ub_), uoff(uoff_), ws(&ws_), o(o_) {}

  char* hreg(int k) const { return ws->up + k * ws->up_bytes; }
  char* dreg(int k) const { return ws->dreg + k * ws->up_bytes; }
  void upload(int k, hipStream_t st) {
    HZ_HIP(hipMemcpyAsync(dreg(k), hreg(k), ws->up_bytes, hipMemcpyHostToDevice, st));
  }
  void read_back(int count, hipStream_t st) {
    HZ_HIP(hipMemcpyAsync(ws->pin, ws->hbuf, size_t(count) * 192 * 16, hipMemcpyDeviceToHost, st));
  }
  void after_sync() {
    for (int i = 0; i < nprob; ++i)
      if (probs[i] && probs[i]->timing) collect_timing(probs[i], false);
  }
  bool finished() const {
    for (const auto& x : S)
      if (!x.done) return false;
    return true;
  }

  // Every solve vacant (finished, nothing to do): a group whose members join later.
  void init_vacant() {
    S.assign(nsol, SolveState());
    for (auto& x : S) x.done = true;
    y.assign(o.restart, cd(0, 0));
  }

  // Starts the solves qs[0 .. nq): ||F||, u = 0, r = F (synchronises).
  hz_status start_slots(const int* qs, int nq, double* const* hist, hipStream_t st) {
    const long N = ws->N, cap = ws->cap;
    const int m = o.restart;
    Region h = region_at(hreg(0), ws->cap);
    const Region d = region_at(dreg(0), ws->cap);
    for (int i = 0; i < nq; ++i) {
      const int q = qs[i];
      h.tab[i] = foff[q];
      h.tab[cap + i] = uoff[q];
      h.tab[2 * cap + i] = long(q) * N;
    }
    upload(0, st);
    launch_mdot_b(Fb, Addr(0, d.tab), 0, 1, nullptr, Fb, Addr(0, d.tab), N, ws->partial,
                  ws->nblk, nq, st);
    launch_reduce_b(ws->partial, ws->nblk, 1, nullptr, ws->hbuf, 192, nq, ws->red, st);
    launch_fill_zero_b(Ub, Addr(0, d.tab + cap), N, nq, st);
    launch_copy_b(Fb, Addr(0, d.tab), ws->RW, Addr(0, d.tab + 2 * cap), N, nq, st);
    read_back(nq, st);
    HZ_HIP(hipStreamSynchronize(st));
    after_sync();
    const auto now = clk::now();
    for (int i = 0; i < nq; ++i) {
      SolveState& x = S[qs[i]];
      x = SolveState();
      x.prob = qs[i] / nrhs;
      x.m = m;
      x.t0 = now;
      x.hist = hist ? hist[qs[i]] : nullptr;
      x.normF = std::sqrt(ws->pin[size_t(i) * 192].x);
      if (!std::isfinite(x.normF)) {
        x.done = true;
        return fail(HZ_EINVAL, "right-hand side is not finite");
      }
      x.H.assign(size_t(m + 1) * m, cd(0, 0));
      x.g.assign(m + 1, cd(0, 0));
      x.cs.assign(m, 0.0);
      x.sn.assign(m, cd(0, 0));
      if (x.normF == 0.0) {
        x.done = true;
        x.conv = true;
        x.est = 0;
        x.true_rel = 0;
        continue;
      }
      x.beta = x.normF;
      x.scale = 1.0 / x.beta;
      x.g[0] = x.beta;
    }
    return HZ_OK;
  }

  hz_status start(double* const* hist, hipStream_t st) {
    t0 = clk::now();
    init_vacant();
    std::vector<int> all(nsol);
    for (int q = 0; q < nsol; ++q) all[q] = q;
    return start_slots(all.data(), nsol, hist, st);
  }

  // The solve in slot q leaves the group (its slot may be started again).
  void vacate(int q) {
    S[q] = SolveState();
    S[q].done = true;
  }

  // Queues one Arnoldi step of every unfinished solve; false when none is left.
  bool issue(hipStream_t st) {
    act.clear();
    for (int q = 0; q < nsol; ++q)
      if (!S[q].done) act.push_back(q);
    issued = !act.empty();
    if (!issued) return false;
    const int na = int(act.size());
    const bool mixed = o.prec == HZ_MIXED;
    const long N = ws->N, cap = ws->cap;
    const long vstr = long(ws->m + 1) * N, zstr = long(ws->m) * N;
    const int p = probs[S[act[0]].prob]->p, nblk = ws->nblk;
    Region h = region_at(hreg(0), ws->cap);
    const Region d = region_at(dreg(0), ws->cap);
    long* t_src = h.tab;               // scale source (r or w) in RW
    long* t_vj = h.tab + cap;          // v_j in V
    long* t_vb = h.tab + 2 * cap;      // basis of the solve in V
    long* t_zj = h.tab + 3 * cap;      // z_j in Z
    long* t_w = h.tab + 4 * cap;       // w in RW
    int maxnv = 0;
    for (int z = 0; z < na; ++z) {
      SolveState& x = S[act[z]];
      const long q = act[z];
      t_src[z] = x.restart ? q * N : (cap + q) * N;
      t_vj[z] = q * vstr + long(x.j) * N;
      t_vb[z] = q * vstr;
      t_zj[z] = q * zstr + long(x.j) * N;
      t_w[z] = (cap + q) * N;
      h.itab[z] = x.j + 1;
      h.scl[z] = x.scale;
      maxnv = std::max(maxnv, x.j + 1);
    }
    // per-solve operators: fine A_eps (coefficients, Jacobi multipliers) and A_0
    zp.resize(na);
    for (int z = 0; z < na; ++z) {
      const hz_problem* pz = probs[S[act[z]].prob];
      zp[z] = S[act[z]].prob;
      h.ptab[z] = mixed ? static_cast<const void*>(pz->fcAe) : static_cast<const void*>(pz->cAe);
      h.ptab[cap + z] = mixed ? static_cast<const void*>(pz->fwdAe) : static_cast<const void*>(pz->wdAe);
      h.ptab[2 * cap + z] = pz->cA0;
    }
    // vectors of this round's projections (a replayed graph must cover every round: 64)
    round_nv = use_graphs() ? 64 : maxnv;
    if (!use_graphs()) {
      enqueue_round(na, st, VC_ALL);
      return true;
    }
    // the launches of a round depend on its problems and their order only (everything that
    // changes from round to round is in the uploaded tables): a repeated round replays a
    // graph captured on its second occurrence
    std::vector<uintptr_t> sig(1, uintptr_t(na));
    for (int z = 0; z < na; ++z) sig.push_back(reinterpret_cast<uintptr_t>(probs[zp[z]]));
    GraphEntry& ge = graphs[sig];
    if (ge.pre) {
      // the coarse solve is a cooperative launch, which stream capture does not take: it
      // runs directly between the two captured halves of the round
      HZ_HIP(hipGraphLaunch(ge.pre, st));
      enqueue_round(na, st, VC_COARSE);
      HZ_HIP(hipGraphLaunch(ge.post, st));
      probs[zp[0]]->stats.graph_rounds += 1;
      return true;
    }
    if (ge.seen++ == 0 || !capture_round(ge, na, st)) enqueue_round(na, st, VC_ALL);
    return true;
  }

  // Graph replay of rounds (HIP stream capture), opt-in with HZ_GRAPHS=1 (measured slower
  // than direct launches for these rounds); off when a member records per-launch device
  // times or after a capture failed.
  struct GraphEntry {
    int seen = 0;
    hipGraphExec_t pre = nullptr, post = nullptr;
  };
  std::map<std::vector<uintptr_t>, GraphEntry> graphs;
  bool graphs_failed = false;

  bool use_graphs() const {
    const char* e = std::getenv("HZ_GRAPHS");
    if (!(e && e[0] == '1') || graphs_failed) return false;
    for (int i = 0; i < nprob; ++i)
      if (probs[i] && probs[i]->timing) return false;
    return true;
  }

  void drop_graphs() {
    for (auto& g : graphs) {
      if (g.second.pre) (void)hipGraphExecDestroy(g.second.pre);
      if (g.second.post) (void)hipGraphExecDestroy(g.second.post);
    }
    graphs.clear();
  }

  // Captures the launches of one half of a round (recording only: nothing runs).
  // Capture runs on a private stream (the caller's may be the null stream, which cannot be
  // captured); only recording happens there, the graphs run on the caller's stream.
  hipStream_t cap_st = nullptr;
  hipGraphExec_t capture_half(int na, int phases, hipStream_t) {
    const char* lg = std::getenv("HZ_GRAPHS_LOG");
    const bool verbose = lg && lg[0] == '1';
    if (!cap_st && hipStreamCreateWithFlags(&cap_st, hipStreamNonBlocking) != hipSuccess) {
      (void)hipGetLastError();
      cap_st = nullptr;
      return nullptr;
    }
    hipStream_t st = cap_st;
    hipError_t e = hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) {
      if (verbose) std::fprintf(stderr, "hz graphs: begin capture: %s\n", hipGetErrorString(e));
      (void)hipGetLastError();
      return nullptr;
    }
    bool ok = true;
    try {
      enqueue_round(na, st, phases);
    } catch (const HipError& he) {
      if (verbose)
        std::fprintf(stderr, "hz graphs: %s during capture: %s\n", he.where.c_str(),
                     hipGetErrorString(he.e));
      ok = false;
    } catch (...) {
      ok = false;
    }
    hipGraph_t g = nullptr;
    e = hipStreamEndCapture(st, &g);
    if (e != hipSuccess) {
      if (verbose) std::fprintf(stderr, "hz graphs: end capture: %s\n", hipGetErrorString(e));
      ok = false;
    }
    hipGraphExec_t ex = nullptr;
    if (ok && g) {
      e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
      if (e != hipSuccess) {
        if (verbose) std::fprintf(stderr, "hz graphs: instantiate: %s\n", hipGetErrorString(e));
        ok = false;
        ex = nullptr;
      }
    }
    if (g) (void)hipGraphDestroy(g);
    (void)hipGetLastError();
    if (!ok && ex) {
      (void)hipGraphExecDestroy(ex);
      ex = nullptr;
    }
    return ex;
  }

  // Captures the two halves of this round around its coarse solve and runs the round from
  // them; false (nothing run) if capture is not available.
  bool capture_round(GraphEntry& ge, int na, hipStream_t st) {
    if (graphs.size() > 32) {              // many distinct member sets: start over
      drop_graphs();
      return false;
    }
    hipGraphExec_t pre = capture_half(na, VC_PRE, st);
    hipGraphExec_t post = pre ? capture_half(na, VC_POST, st) : nullptr;
    if (!pre || !post) {
      if (pre) (void)hipGraphExecDestroy(pre);
      graphs_failed = true;
      drop_graphs();
      return false;
    }
    ge.pre = pre;
    ge.post = post;
    HZ_HIP(hipGraphLaunch(pre, st));
    enqueue_round(na, st, VC_COARSE);
    HZ_HIP(hipGraphLaunch(post, st));
    return true;
  }

  // Upload of this round's tables, the round's kernels and the read-back (as built by
  // issue()).
  void enqueue_round(int na, hipStream_t st, int phases) {
    const bool mixed = o.prec == HZ_MIXED;
    const long N = ws->N, cap = ws->cap;
    const int p = probs[zp[0]]->p, nblk = ws->nblk;
    const Region d = region_at(dreg(0), ws->cap);
    if (phases & VC_PRE) upload(0, st);
    const long* d_src = d.tab;
    const long* d_vj = d.tab + cap;
    const long* d_vb = d.tab + 2 * cap;
    const long* d_zj = d.tab + 3 * cap;
    const long* d_w = d.tab + 4 * cap;
    // v_j = r / beta (cycle start) or w / h_{j,j-1}
    if (phases & VC_PRE) launch_scale_b(ws->RW, Addr(0, d_src), d.scl, ws->V, Addr(0, d_vj), N, na, st);
    // z_j = V-cycle(v_j) for every unfinished solve at once
    hz_problem* pr0 = probs[zp[0]];
    if (!mixed) {
      DevOp<double> fine{nullptr, nullptr, pr0->M,
                         reinterpret_cast<const double2* const*>(d.ptab),
                         reinterpret_cast<const double2* const*>(d.ptab + cap)};
      fine.pn = pr0->cells;
      vcycle_group<double>(probs, zp.data(), na, fine, pr0->rw, ws->s64,
                           static_cast<double2*>(ws->gb), ws->V, Addr(0, d_vj), ws->Zd,
                           Addr(0, d_zj), st, phases);
    } else {
      DevOp<float> fine{nullptr, nullptr, pr0->M,
                        reinterpret_cast<const float2* const*>(d.ptab),
                        reinterpret_cast<const float2* const*>(d.ptab + cap)};
      fine.pn = pr0->cells;
      if (phases & VC_PRE) launch_d2f_b(ws->V, Addr(0, d_vj), ws->s32.ff, Addr(N), N, na, st);
      vcycle_group<float>(probs, zp.data(), na, fine, pr0->frw, ws->s32,
                          static_cast<float2*>(ws->gb), ws->s32.ff, Addr(N), ws->Zf,
                          Addr(0, d_zj), st, phases);
    }
    if (!(phases & VC_POST)) return;
    // w = A_0 z_j
    DevOp<double> a0{nullptr, nullptr, pr0->M, reinterpret_cast<const double2* const*>(d.ptab + 2 * cap),
                     nullptr};
    a0.pn = pr0->cells;
    apply_a0(a0, p, Addr(0, d_zj), Addr(0, d_w), na, st);
    // CGS2: two passes of h = V^H w, w -= V h; then |w|^2
    // (the first pass's update and the second pass's projection share one read of V)
    launch_mdot_b(ws->V, Addr(0, d_vb), N, 64, d.itab, ws->RW, Addr(0, d_w), N, ws->partial, nblk, na, st);
    launch_reduce_b(ws->partial, nblk, 64, d.itab, ws->hbuf, 192, na, ws->red, st);
    launch_maxpy_mdot_b(ws->V, Addr(0, d_vb), N, round_nv, d.itab, ws->hbuf, 192, ws->RW,
                        Addr(0, d_w), N, ws->partial, na, st);
    launch_reduce_b(ws->partial, fused_blocks(N), 64, d.itab, ws->hbuf + 64, 192, na, ws->red, st);
    launch_maxpy_b(ws->V, Addr(0, d_vb), N, round_nv, d.itab, ws->hbuf + 64, 192, ws->RW,
                   Addr(0, d_w), N, ws->partial, na, st);
    launch_reduce_b(ws->partial, fused_blocks(N), 1, nullptr, ws->hbuf + 128, 192, na, ws->red, st);
    read_back(na, st);
  }

  void apply_a0(const DevOp<double>& a0, int p, Addr az, Addr aw, int nb, hipStream_t st) {
    if (o.prec != HZ_MIXED)
      launch_stencil<double, double, double, double>(p, ST_APPLY, a0, ws->Zd, az, nullptr, Addr(),
                                                     ws->RW, aw, nb, st);
    else
      launch_stencil<double, float, double, double>(p, ST_APPLY, a0, ws->Zf, az, nullptr, Addr(),
                                                    ws->RW, aw, nb, st);
  }

  // After the round's read-back has landed (the caller synchronised the stream).
  hz_status complete(hipStream_t st) {
    if (!issued) return HZ_OK;
    issued = false;
    after_sync();
    const int na = int(act.size());
    const int m = o.restart;
    end.clear();
    for (int z = 0; z < na; ++z) {
      SolveState& x = S[act[z]];
      const double2* hb = ws->pin + size_t(z) * 192;
      const int j = x.j;
      x.its += 1;
      for (int i = 0; i <= j; ++i)
        x.Hat(i, j) = (cd(0, 0) + cd(hb[i].x, hb[i].y)) + cd(hb[64 + i].x, hb[64 + i].y);
      const double hnext = std::sqrt(hb[128].x);
      if (!std::isfinite(hnext)) return fail(HZ_EDEVICE, "non-finite Arnoldi norm");
      x.Hat(j + 1, j) = hnext;
      for (int i = 0; i < j; ++i) {
        const cd a = x.Hat(i, j), b = x.Hat(i + 1, j);
        x.Hat(i, j) = x.cs[i] * a + x.sn[i] * b;
        x.Hat(i + 1, j) = -std::conj(x.sn[i]) * a + x.cs[i] * b;
      }
      givens(x.Hat(j, j), x.Hat(j + 1, j), x.cs[j], x.sn[j]);
      {
        const cd a = x.Hat(j, j), b = x.Hat(j + 1, j);
        x.Hat(j, j) = x.cs[j] * a + x.sn[j] * b;
        x.Hat(j + 1, j) = 0;
      }
      x.g[j + 1] = -std::conj(x.sn[j]) * x.g[j];
      x.g[j] = x.cs[j] * x.g[j];
      x.est = std::abs(x.g[j + 1]) / x.normF;
      if (x.hist) x.hist[x.its - 1] = x.est;
      if (x.est <= o.tol || x.its >= o.maxit || hnext == 0.0 || j + 1 == m) {
        end.push_back(act[z]);
      } else {
        x.restart = false;
        x.scale = 1.0 / hnext;
        x.j = j + 1;
      }
    }
    if (end.empty()) return HZ_OK;
    // ---- cycle ends: u += Z y, r = F - A_0 u, ||r|| ----
    const bool mixed = o.prec == HZ_MIXED;
    const long N = ws->N, cap = ws->cap;
    const long zstr = long(ws->m) * N;
    const int ne = int(end.size());
    Region h2 = region_at(hreg(1), ws->cap);
    const Region d2 = region_at(dreg(1), ws->cap);
    for (int e = 0; e < ne; ++e) {
      SolveState& x = S[end[e]];
      const long q = end[e];
      const int jend = x.j + 1;
      for (int i = jend - 1; i >= 0; --i) {
        cd acc = x.g[i];
        for (int l = i + 1; l < jend; ++l) acc -= x.Hat(i, l) * y[l];
        y[i] = acc / x.Hat(i, i);
      }
      for (int i = 0; i < jend; ++i) h2.y[size_t(e) * 64 + i] = make_double2(y[i].real(), y[i].imag());
      h2.tab[e] = q * zstr;
      h2.tab[cap + e] = uoff[q];
      h2.tab[2 * cap + e] = foff[q];
      h2.tab[3 * cap + e] = q * N;
      h2.itab[e] = jend;
      h2.ptab[e] = probs[x.prob]->cA0;
    }
    upload(1, st);
    if (!mixed)
      launch_update_b<double>(ws->Zd, Addr(0, d2.tab), N, 64, d2.itab, d2.y, 64, Ub,
                              Addr(0, d2.tab + cap), N, ne, st);
    else
      launch_update_b<float>(ws->Zf, Addr(0, d2.tab), N, 64, d2.itab, d2.y, 64, Ub,
                             Addr(0, d2.tab + cap), N, ne, st);
    // r = F - A_0 u (each solve with its own A_0)
    {
      const hz_problem* pe = probs[S[end[0]].prob];
      DevOp<double> a0{nullptr, nullptr, pe->M,
                       reinterpret_cast<const double2* const*>(d2.ptab), nullptr};
      a0.pn = pe->cells;
      launch_stencil<double, double, double, double>(pe->p, ST_RESID, a0, Ub,
                                                     Addr(0, d2.tab + cap), Fb,
                                                     Addr(0, d2.tab + 2 * cap), ws->RW,
                                                     Addr(0, d2.tab + 3 * cap), ne, st);
    }
    launch_mdot_b(ws->RW, Addr(0, d2.tab + 3 * cap), 0, 1, nullptr, ws->RW, Addr(0, d2.tab + 3 * cap),
                  N, ws->partial, ws->nblk, ne, st);
    launch_reduce_b(ws->partial, ws->nblk, 1, nullptr, ws->hbuf, 192, ne, ws->red, st);
    read_back(ne, st);
    HZ_HIP(hipStreamSynchronize(st));
    after_sync();
    for (int e = 0; e < ne; ++e) {
      SolveState& x = S[end[e]];
      x.beta = std::sqrt(ws->pin[size_t(e) * 192].x);
      x.true_rel = x.beta / x.normF;
      if (x.true_rel <= o.tol) {
        x.done = true;
        x.conv = true;
      } else if (x.its >= o.maxit) {
        x.done = true;
      } else {
        x.restart = true;
        x.j = 0;
        x.scale = 1.0 / x.beta;
        std::fill(x.H.begin(), x.H.end(), cd(0, 0));
        std::fill(x.g.begin(), x.g.end(), cd(0, 0));
        x.g[0] = x.beta;
      }
    }
    return HZ_OK;
  }

  hz_status check_device() {
    for (int i = 0; i < nprob; ++i) {
      if (!probs[i]) continue;
      int e = 0;
      HZ_HIP(hipMemcpy(&e, probs[i]->cw.err, sizeof(int), hipMemcpyDeviceToHost));
      if (e) return fail(HZ_EDEVICE, "coarse solve: a wait for another workgroup timed out");
    }
    return HZ_OK;
  }

  hz_result result_of(int q) const {
    hz_result r{};
    r.iterations = S[q].its;
    r.converged = S[q].conv ? 1 : 0;
    r.rel_res_true = S[q].true_rel;
    r.rel_res_est = S[q].est;
    r.setup_s = probs[S[q].prob] ? probs[S[q].prob]->setup_s : 0.0;
    r.solve_s = secs(S[q].t0);
    return r;
  }
  void results(hz_result* res) const {
    for (int q = 0; q < nsol; ++q) res[q] = result_of(q);
  }
};

hz_status lockstep(hz_problem* const* probs, int nprob, int nrhs, const double2* Fb,
                   const long* foff, double2* Ub, const long* uoff, Workspace& ws,
                   const hz_options& o, hz_result* res, double* const* hist, hipStream_t st) {
  Lockstep L(probs, nprob, nrhs, Fb, foff, Ub, uoff, ws, o);
  hz_status r = L.start(hist, st);
  if (r != HZ_OK) return r;
  while (L.issue(st)) {
    HZ_HIP(hipStreamSynchronize(st));
    r = L.complete(st);
    if (r != HZ_OK) return r;
  }
  r = L.check_device();
  if (r != HZ_OK) return r;
  if (res) L.results(res);
  return HZ_OK;
}

hz_status solve_impl(hz_problem* pr, const double2* F, double2* u, const hz_options& o,
                     hz_result* res, double* hist, hipStream_t st) {
  const bool mixed = o.prec == HZ_MIXED;
  if (o.restart > pr->m) return fail(HZ_EINVAL, "restart exceeds the capacity given at creation");
  if (mixed) ensure_mixed_work(pr, st);
  else {
    if (!pr->S) return fail(HZ_EINVAL, "problem was created for mixed precision only");
    ensure_fp64_work(pr);
  }
  if (!pr->ws1 || pr->ws1->prec != o.prec) {
    pr->ws1.reset();
    pr->ws1 = make_workspace(1, pr->m, o.prec, pr->N, pr->Nc, pr->G, 0, false);
    pr->ws1->s64 = pr->s64;
    pr->ws1->s32 = pr->s32;
    pr->ws1->gb = pr->cw.g;
  }
  const long off = 0;
  hz_problem* const probs[1] = {pr};
  double* const hists[1] = {hist};
  return lockstep(probs, 1, 1, F, &off, u, &off, *pr->ws1, o, res, hists, st);
}

}  // namespace

// =========================================================================================
// C ABI
// =========================================================================================

// ------------------------------------------------------------------------------------------
// hz_apply and its allocation-free variant share one body; they differ only in where the
// scratch of the kernels lives (the problem's own buffers, allocated on first use, or the
// file-scope device array below).
// ------------------------------------------------------------------------------------------

namespace {

struct ApplyBufs {
  Scratch<double> s64;                 // V-cycle iterates, residual, coarse vectors (FP64)
  Scratch<float> s32;                  // the same in FP32, plus the FP32 copy of the input
  float2 *ax32 = nullptr, *af32 = nullptr, *ay32 = nullptr;   // FP32 staging of x, f, y (fine)
  float2 *cx32 = nullptr, *cy32 = nullptr;                    // and of coarse x, y
  CoarseSolveWork cw;                  // coarse forward-sweep buffer and timeout flag
  bool own = true;                     // the problem's own buffers (timed coarse solves)
};

hz_status check_apply(hz_problem* pr, int op, const hz_c64* d_x, const hz_c64* d_f,
                      const hz_c64* d_y, int prec) {
  if (!pr || !d_x || !d_y) return fail(HZ_EINVAL, "null argument");
  if ((op == HZ_OP_JACOBI || op == HZ_OP_RESID_RESTRICT) && !d_f)
    return fail(HZ_EINVAL, "this operator needs d_f");
  if (op < 0 || op > HZ_OP_RESID_RESTRICT) return fail(HZ_EINVAL, "unknown operator");
  if (prec != HZ_FP64 && prec != HZ_MIXED) return fail(HZ_EINVAL, "bad precision");
  if (prec == HZ_FP64 && !pr->S) return fail(HZ_EINVAL, "problem was created for mixed precision only");
  return HZ_OK;
}

void apply_impl(hz_problem* pr, int op, const double2* x, const double2* f, double2* y, int prec,
                const ApplyBufs& b, hipStream_t st) {
  const int p = pr->p;
  const bool fine_in = !(op == HZ_OP_PROLONG || op == HZ_OP_COARSE_SOLVE || op == HZ_OP_COARSE_A);
  const bool fine_out = !(op == HZ_OP_RESTRICT || op == HZ_OP_COARSE_SOLVE ||
                          op == HZ_OP_COARSE_A || op == HZ_OP_RESID_RESTRICT);
  const Addr o;
  if (prec == HZ_FP64) {
    Level<double> lv = level64(pr, b.s64);
    lv.cw = b.cw;
    DevOp<double> a0{pr->cA0, nullptr, pr->M};
    a0.pn = pr->cells;
    switch (op) {
      case HZ_OP_A0: launch_stencil<double, double, double, double>(p, ST_APPLY, a0, x, o, nullptr, o, y, o, 1, st); break;
      case HZ_OP_AEPS: launch_stencil<double, double, double, double>(p, ST_APPLY, lv.fine, x, o, nullptr, o, y, o, 1, st); break;
      case HZ_OP_JACOBI: launch_stencil<double, double, double, double>(p, ST_SMOOTH, lv.fine, x, o, f, o, y, o, 1, st); break;
      case HZ_OP_RESTRICT: launch_restrict<double>(p, pr->M, pr->Mc, pr->rw, x, y, 1, o, o, st); break;
      case HZ_OP_PROLONG: launch_prolong<double>(p, pr->M, pr->Mc, pr->rw, x, y, false, 1, o, o, st); break;
      case HZ_OP_VCYCLE: vcycle<double>(pr, lv, x, y, st, b.own); break;
      case HZ_OP_COARSE_SOLVE: timed_coarse_solve<double>(pr, lv, x, y, st, b.own); break;
      case HZ_OP_COARSE_A: launch_stencil<double, double, double, double>(p, ST_APPLY, lv.coarse, x, o, nullptr, o, y, o, 1, st); break;
      case HZ_OP_RESID_RESTRICT:
        if (launch_resid_restrict<double>(p, lv.fine, x, o, f, o, pr->Mc, pr->rw, y, o, 1, st)) break;
        launch_stencil<double, double, double, double>(p, ST_RESID, lv.fine, x, o, f, o, b.s64.rf, o, 1, st);
        launch_restrict<double>(p, pr->M, pr->Mc, pr->rw, b.s64.rf, y, 1, o, o, st);
        break;
    }
    return;
  }
  Level<float> lv = level32(pr, b.s32);
  lv.cw = b.cw;
  const long nin = fine_in ? pr->N : pr->Nc;
  const long nout = fine_out ? pr->N : pr->Nc;
  // FP32 copies: x -> ax32 (fine) or cx32 (coarse), f -> af32; result in ay32 / cy32
  float2* xin = fine_in ? b.ax32 : b.cx32;
  launch_d2f(x, xin, nin, st);
  if (f) launch_d2f(f, b.af32, pr->N, st);
  float2* yout = fine_out ? b.ay32 : b.cy32;
  switch (op) {
    case HZ_OP_A0: {
      DevOp<double> a0{pr->cA0, nullptr, pr->M};
      a0.pn = pr->cells;
      launch_stencil<double, float, double, double>(p, ST_APPLY, a0, xin, o, nullptr, o, y, o, 1, st);
      return;
    }
    case HZ_OP_AEPS: launch_stencil<float, float, float, float>(p, ST_APPLY, lv.fine, xin, o, nullptr, o, yout, o, 1, st); break;
    case HZ_OP_JACOBI: launch_stencil<float, float, float, float>(p, ST_SMOOTH, lv.fine, xin, o, b.af32, o, yout, o, 1, st); break;
    case HZ_OP_RESTRICT: launch_restrict<float>(p, pr->M, pr->Mc, pr->frw, xin, yout, 1, o, o, st); break;
    case HZ_OP_PROLONG: launch_prolong<float>(p, pr->M, pr->Mc, pr->frw, xin, yout, false, 1, o, o, st); break;
    case HZ_OP_VCYCLE: vcycle<float>(pr, lv, xin, yout, st, b.own); break;
    case HZ_OP_COARSE_SOLVE: timed_coarse_solve<float>(pr, lv, xin, yout, st, b.own); break;
    case HZ_OP_COARSE_A: launch_stencil<float, float, float, float>(p, ST_APPLY, lv.coarse, xin, o, nullptr, o, yout, o, 1, st); break;
    case HZ_OP_RESID_RESTRICT:
      if (launch_resid_restrict<float>(p, lv.fine, xin, o, b.af32, o, pr->Mc, pr->frw, yout, o, 1, st))
        break;
      launch_stencil<float, float, float, float>(p, ST_RESID, lv.fine, xin, o, b.af32, o, b.s32.rf, o, 1, st);
      launch_restrict<float>(p, pr->M, pr->Mc, pr->frw, b.s32.rf, yout, 1, o, o, st);
      break;
  }
  launch_f2d(yout, y, nout, st);
}

}  // namespace

// Scratch of hz_apply_noalloc: one array per device (each GPU holds its own copy at its own
// address until the process ends). Host code never uses its name as an address: the device
// address is looked up once per device with hipGetSymbolAddress and kept in g_scratch_ptr.
constexpr size_t kScratchBytes = size_t(64) << 20;
static __device__ __align__(256) char scratch[kScratchBytes];

namespace {

std::mutex g_scratch_mu;
std::map<int, char*> g_scratch_ptr;

// Device address of the current device's scratch array (set up on the first call per device,
// with that device current; also creates the device's coarse-solve ordering event then).
char* noalloc_scratch() {
  int dev = 0;
  HZ_HIP(hipGetDevice(&dev));
  std::lock_guard<std::mutex> g(g_scratch_mu);
  auto it = g_scratch_ptr.find(dev);
  if (it != g_scratch_ptr.end()) return it->second;
  void* ptr = nullptr;
  const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !ptr) throw HipError{e, "hipGetSymbolAddress(scratch)"};
  coarse_order_init(dev);
  g_scratch_ptr[dev] = static_cast<char*>(ptr);
  return static_cast<char*>(ptr);
}

// Carves the buffers of one apply out of the scratch array (256-byte aligned pieces).
struct Carver {
  char* base;
  size_t off = 0;
  template <typename T> T* take(size_t n) {
    T* p = reinterpret_cast<T*>(base + off);
    off += (n * sizeof(T) + 255) / 256 * 256;
    return p;
  }
};
ApplyBufs noalloc_carve(char* base, long N, long Nc, long G, int prec, size_t* used) {
  Carver c{base};
  ApplyBufs b;
  b.cw.err = c.take<int>(64);
  b.cw.g = c.take<double2>(size_t(G));
  if (prec == HZ_FP64) {
    b.s64.cap = 1;
    b.s64.ua = c.take<double2>(N);
    b.s64.ub = c.take<double2>(N);
    b.s64.rf = c.take<double2>(N);
    b.s64.rc = c.take<double2>(Nc);
    b.s64.ec = c.take<double2>(Nc);
  } else {
    b.s32.cap = 1;
    b.s32.ua = c.take<float2>(N);
    b.s32.ub = c.take<float2>(N);
    b.s32.rf = c.take<float2>(N);
    b.s32.ff = c.take<float2>(N);
    b.s32.rc = c.take<float2>(Nc);
    b.s32.ec = c.take<float2>(Nc);
    b.ax32 = c.take<float2>(N);
    b.af32 = c.take<float2>(N);
    b.ay32 = c.take<float2>(N);
    b.cx32 = c.take<float2>(Nc);
    b.cy32 = c.take<float2>(Nc);
  }
  if (used) *used = c.off;
  return b;
}
size_t noalloc_bytes(long N, long Nc, long G, int prec) {
  size_t used = 0;
  (void)noalloc_carve(nullptr, N, Nc, G, prec, &used);
  return used;
}
ApplyBufs noalloc_layout(char* base, long N, long Nc, long G, int prec) {
  return noalloc_carve(base, N, Nc, G, prec, nullptr);
}

}  // namespace

extern "C" {

hz_status hz_default_options(hz_options* o) {
  if (!o) return fail(HZ_EINVAL, "null options");
  o->nu = 2;
  o->omega = 0.6;
  o->restart = 50;
  o->maxit = 5000;
  o->tol = 1e-8;
  o->prec = HZ_FP64;
  o->timing = 0;
  return HZ_OK;
}

const char* hz_last_error(void) { return g_err.c_str(); }

size_t hz_footprint_estimate(double k, double h, int p, const hz_options* o) {
  hz_options d;
  hz_default_options(&d);
  const hz_options& oo = o ? *o : d;
  int n = 0;
  std::string why;
  if (!valid_problem(k, h, p, cd(1, 1), n, why) || !valid_options(oo, why)) return 0;
  return resident_bytes(n, p, oo.restart, oo.prec);
}

namespace {
hz_status finish_create(hz_problem* pr, hipStream_t st, clk::time_point t0, hz_problem** out);
}

hz_status hz_create_problem(double k, double h, int p, hz_c64 s, const hz_options* o,
                            void* hip_stream, hz_problem** out) {
  if (!out) return fail(HZ_EINVAL, "null output pointer");
  *out = nullptr;
  hz_options opt;
  hz_default_options(&opt);
  if (o) opt = *o;
  int n = 0;
  std::string why;
  const cd sc(s.re, s.im);
  if (!valid_problem(k, h, p, sc, n, why) || !valid_options(opt, why)) return fail(HZ_EINVAL, why);
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  const auto t0 = clk::now();
  hz_problem* pr = nullptr;
  try {
    pr = new hz_problem();
    pr->k = k; pr->n = n; pr->p = p; pr->s = sc; pr->opt = opt;
    pr->M = p * n + 1;
    pr->Mc = p * (n / 2) + 1;
    pr->N = long(pr->M) * pr->M;
    pr->Nc = long(pr->Mc) * pr->Mc;
    pr->L = CoarseLayout{p, n / 2, pr->Mc};
    pr->m = opt.restart;
    upload_tables(pr, st);
    return finish_create(pr, st, t0, out);
  } catch (...) {
    delete pr;
    return map_exception();
  }
}

hz_status hz_create_problem_cells(const double* k_cell, const hz_c64* s_cell, double h, int p,
                                  const hz_options* o, void* hip_stream, hz_problem** out) {
  if (!out) return fail(HZ_EINVAL, "null output pointer");
  *out = nullptr;
  if (!k_cell || !s_cell) return fail(HZ_EINVAL, "null cell array");
  hz_options opt;
  hz_default_options(&opt);
  if (o) opt = *o;
  int n = 0;
  std::string why;
  if (!valid_problem(1.0, h, p, cd(1, 1), n, why) || !valid_options(opt, why)) return fail(HZ_EINVAL, why);
  double kmax = 0.0;
  for (long c = 0; c < long(n) * n; ++c) {
    const double kv = k_cell[c];
    const cd sv(s_cell[c].re, s_cell[c].im);
    if (!(kv > 0) || !std::isfinite(kv))
      return fail(HZ_EINVAL, "k_cell[" + std::to_string(c) + "] must be finite and > 0");
    if (!std::isfinite(sv.real()) || !std::isfinite(sv.imag()) || !(sv.imag() > 0))
      return fail(HZ_EINVAL, "s_cell[" + std::to_string(c) + "] must be finite with Im(s) > 0");
    kmax = std::max(kmax, kv);
  }
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  const auto t0 = clk::now();
  hz_problem* pr = nullptr;
  try {
    pr = new hz_problem();
    pr->k = kmax; pr->n = n; pr->p = p; pr->s = cd(0, 0); pr->opt = opt;
    pr->cells = 1;
    pr->M = p * n + 1;
    pr->Mc = p * (n / 2) + 1;
    pr->N = long(pr->M) * pr->M;
    pr->Nc = long(pr->Mc) * pr->Mc;
    pr->L = CoarseLayout{p, n / 2, pr->Mc};
    pr->m = opt.restart;
    upload_tables(pr, st);
    upload_cells(pr, k_cell, s_cell, st);
    return finish_create(pr, st, t0, out);
  } catch (...) {
    delete pr;
    return map_exception();
  }
}

namespace {

// Coarse factor, coarse-solve buffers and V-cycle scratch of a problem whose operators are
// on the device; deletes pr on failure.
hz_status finish_create(hz_problem* pr, hipStream_t st, clk::time_point t0, hz_problem** out) {
  const hz_options& opt = pr->opt;
  try {
    // coarse factor (FP64), then the FP32 copy for mixed-precision problems
    {
      const Sizes z = sizes_of(pr->n, pr->p);
      pr->G = z.G;
      pr->fel = z.factor_elems;
    }
    if (use_mf()) {
      pr->sym = &mf_symbolic(pr->p, pr->n / 2);
      upload_symbolic(pr, st);
    }
    pr->S = opt.prec == HZ_MIXED ? pr->mem.alloc_async<double2>(pr->fel, st)
                                 : pr->mem.alloc<double2>(pr->fel);
    {
      DevOp<double> cop{pr->cAc, nullptr, pr->Mc};
      cop.pn = pr->cells;
      pr->timing = opt.timing != 0;
      hipEvent_t f0 = nullptr, f1 = nullptr;
      if (pr->timing) {
        HZ_HIP(hipEventCreate(&f0));
        HZ_HIP(hipEventCreate(&f1));
        HZ_HIP(hipEventRecord(f0, st));
      }
      hz_status fs;
      if (pr->sym) {
        int* flag = pr->mem.alloc_async<int>(1, st);
        fs = mf_factor(*pr->sym, cop, pr->S, flag, st);
        pr->mem.release_async(flag, st);
      } else {
        CoarseFactorWork wk;
        const size_t mb = size_t(pr->L.size(0));
        wk.T = pr->mem.alloc_async<double2>(2 * mb * mb, st);     // one set per chain
        wk.W = pr->mem.alloc_async<double2>(2 * sweep_panel_elems(mb), st);
        wk.R = pr->mem.alloc_async<double2>(2 * sweep_pinv_elems(), st);
        wk.flag = pr->mem.alloc_async<int>(1, st);
        fs = coarse_factor(pr->L, cop, pr->S, wk, st);
        pr->mem.release_async(wk.T, st);
        pr->mem.release_async(wk.W, st);
        pr->mem.release_async(wk.R, st);
        pr->mem.release_async(wk.flag, st);
      }
      if (pr->timing) {
        HZ_HIP(hipEventRecord(f1, st));
        HZ_HIP(hipEventSynchronize(f1));
        float ms = 0;
        HZ_HIP(hipEventElapsedTime(&ms, f0, f1));
        pr->stats.factor_ms = ms;
        (void)hipEventDestroy(f0);
        (void)hipEventDestroy(f1);
      }
      if (fs != HZ_OK) {
        delete pr;
        return fail(fs, "zero or non-finite pivot in the coarse factorisation");
      }
      pr->stats.factor_flop = pr->sym ? pr->sym->flop : band_factor_flop(pr->L);
    }
    pr->cw.g = pr->mem.alloc<double2>(4 * size_t(pr->G));
    pr->cw.err = pr->mem.alloc<int>(64);
    HZ_HIP(hipMemsetAsync(pr->cw.err, 0, 64 * sizeof(int), st));
    {
      const char* env = std::getenv("HZ_COARSE_PERSISTENT");
      pr->cw.persistent = !(env && env[0] == '0');
    }
    if (opt.prec == HZ_MIXED) {
      ensure_mixed_work(pr, st);
      pr->mem.release_async(pr->S, st);
      pr->S = nullptr;
    } else {
      ensure_fp64_work(pr);
    }
    HZ_HIP(hipStreamSynchronize(st));
    // set-up temporaries went back to the device's stream-ordered pool (the FP64 factor of a
    // mixed problem is the largest); hand the unused part back so that later allocations,
    // of this or any other problem, find it
    {
      int dev = 0;
      hipMemPool_t pool = nullptr;
      if (hipGetDevice(&dev) == hipSuccess && hipDeviceGetDefaultMemPool(&pool, dev) == hipSuccess)
        (void)hipMemPoolTrimTo(pool, 0);
      (void)hipGetLastError();
    }
    pr->setup_s = secs(t0);
    *out = pr;
    return HZ_OK;
  } catch (...) {
    delete pr;
    return map_exception();
  }
}

}  // namespace

hz_status hz_problem_info(const hz_problem* pr, long* n_dofs, long* n_coarse, size_t* footprint) {
  if (!pr) return fail(HZ_EINVAL, "null problem");
  if (n_dofs) *n_dofs = pr->N;
  if (n_coarse) *n_coarse = pr->Nc;
  if (footprint) *footprint = pr->mem.bytes;
  return HZ_OK;
}

hz_status hz_planewave_rhs(const hz_problem* pr, double theta, hz_c64* d_F, void* hip_stream) {
  if (!pr || !d_F) return fail(HZ_EINVAL, "null argument");
  if (!std::isfinite(theta)) return fail(HZ_EINVAL, "theta must be finite");
  try {
    launch_planewave(pr->p, pr->n, pr->k, theta, pr->gl_t, pr->gl_w, pr->lag,
                     reinterpret_cast<double2*>(d_F), static_cast<hipStream_t>(hip_stream));
    return HZ_OK;
  } catch (...) {
    return map_exception();
  }
}

hz_status hz_gaussian_rhs(const hz_problem* pr, double sx, double sy, double amp, double width,
                          hz_c64* d_F, void* hip_stream) {
  if (!pr || !d_F) return fail(HZ_EINVAL, "null argument");
  if (!std::isfinite(sx) || !std::isfinite(sy) || !std::isfinite(amp) || !(width >= 0) ||
      !std::isfinite(width))
    return fail(HZ_EINVAL, "source centre and amplitude must be finite, width finite and >= 0");
  try {
    const double* q = pr->qtab;
    launch_gauss_rhs(pr->p, pr->n, sx, sy, amp, width, q, q + pr->nq, q + 2 * pr->nq,
                     q + 3 * pr->nq, pr->qloc, pr->nq, reinterpret_cast<double2*>(d_F),
                     static_cast<hipStream_t>(hip_stream));
    return HZ_OK;
  } catch (...) {
    return map_exception();
  }
}

hz_status hz_solve(hz_problem* pr, const hz_c64* d_F, hz_c64* d_u, const hz_options* o,
                   hz_result* res, double* h_res_hist, void* hip_stream) {
  if (!pr || !d_F || !d_u) return fail(HZ_EINVAL, "null argument");
  hz_options opt = pr->opt;
  if (o) {
    opt.restart = o->restart;
    opt.maxit = o->maxit;
    opt.tol = o->tol;
    opt.prec = o->prec;
  }
  std::string why;
  if (!valid_options(opt, why)) return fail(HZ_EINVAL, why);
  BusyGuard guard(pr->busy);
  if (!guard.ok) return fail(HZ_EBUSY, "problem is in use");
  try {
    return solve_impl(pr, reinterpret_cast<const double2*>(d_F), reinterpret_cast<double2*>(d_u),
                      opt, res, h_res_hist, static_cast<hipStream_t>(hip_stream));
  } catch (...) {
    return map_exception();
  }
}

hz_status hz_apply(const hz_problem* cpr, int op, const hz_c64* d_x, const hz_c64* d_f,
                   hz_c64* d_y, int prec, void* hip_stream) {
  hz_problem* pr = const_cast<hz_problem*>(cpr);
  hz_status v = check_apply(pr, op, d_x, d_f, d_y, prec);
  if (v != HZ_OK) return v;
  BusyGuard guard(pr->busy);
  if (!guard.ok) return fail(HZ_EBUSY, "problem is in use");
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  try {
    ApplyBufs b;
    if (prec == HZ_FP64) {
      ensure_fp64_work(pr);
      b.s64 = pr->s64;
    } else {
      ensure_mixed_work(pr, st);
      ensure_apply32(pr);
      b.s32 = pr->s32;
      b.ax32 = pr->ax32; b.af32 = pr->af32; b.ay32 = pr->ay32;
      b.cx32 = pr->cx32; b.cy32 = pr->cy32;
    }
    b.cw = pr->cw;
    b.own = true;
    apply_impl(pr, op, reinterpret_cast<const double2*>(d_x), reinterpret_cast<const double2*>(d_f),
               reinterpret_cast<double2*>(d_y), prec, b, st);
    return HZ_OK;
  } catch (...) {
    return map_exception();
  }
}

hz_status hz_apply_noalloc(const hz_problem* cpr, int op, const hz_c64* d_x, const hz_c64* d_f,
                           hz_c64* d_y, int prec, void* hip_stream) {
  hz_problem* pr = const_cast<hz_problem*>(cpr);
  hz_status v = check_apply(pr, op, d_x, d_f, d_y, prec);
  if (v != HZ_OK) return v;
  if (prec == HZ_MIXED && !pr->Sf)
    return fail(HZ_EINVAL, "the problem holds no FP32 coarse factor (create it with HZ_MIXED, or "
                           "run one mixed-precision hz_apply or hz_solve first)");
  const size_t need = noalloc_bytes(pr->N, pr->Nc, pr->G, prec);
  if (need > kScratchBytes)
    return fail(HZ_EINVAL, "the allocation-free apply needs " + std::to_string(need) +
                               " scratch bytes for this problem; its maximum is " +
                               std::to_string(kScratchBytes));
  BusyGuard guard(pr->busy);
  if (!guard.ok) return fail(HZ_EBUSY, "problem is in use");
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  try {
    char* base = noalloc_scratch();
    ApplyBufs b = noalloc_layout(base, pr->N, pr->Nc, pr->G, prec);
    b.cw.persistent = pr->cw.persistent;
    b.own = false;
    // the coarse solve's timeout flag must start at zero (the array keeps the last call's
    // contents); a fill kernel, not a memset, so that the call may be captured
    launch_fill_zero(reinterpret_cast<double2*>(b.cw.err), 16, st);
    set_stencil_tuning(false);
    struct Restore { ~Restore() { set_stencil_tuning(true); } } restore;
    apply_impl(pr, op, reinterpret_cast<const double2*>(d_x), reinterpret_cast<const double2*>(d_f),
               reinterpret_cast<double2*>(d_y), prec, b, st);
    return HZ_OK;
  } catch (...) {
    return map_exception();
  }
}

hz_status hz_solve_batched(hz_problem* const* probs, int nprob, const hz_c64* const* d_F,
                           int nrhs_per_prob, hz_c64* const* d_u, const hz_options* o,
                           hz_result* res, void* hip_stream) {
  if (!probs || nprob < 1 || nrhs_per_prob < 1 || !d_F || !d_u) return fail(HZ_EINVAL, "bad arguments");
  const long nsol = long(nprob) * nrhs_per_prob;
  if (nsol > 4096) return fail(HZ_EINVAL, "at most 4096 solves per batch");
  for (int i = 0; i < nprob; ++i) {
    if (!probs[i]) return fail(HZ_EINVAL, "null problem");
    if (probs[i]->n != probs[0]->n || probs[i]->p != probs[0]->p)
      return fail(HZ_EINVAL, "batched problems must share (h, p)");
    if (probs[i]->cells != probs[0]->cells)
      return fail(HZ_EINVAL, "batched problems must all have constant k or all per-cell k");
    if (probs[i]->opt.nu != probs[0]->opt.nu)
      return fail(HZ_EINVAL, "batched problems must share nu");
    for (int i2 = 0; i2 < i; ++i2)
      if (probs[i2] == probs[i]) return fail(HZ_EINVAL, "a problem appears twice in the batch");
  }
  for (long q = 0; q < nsol; ++q)
    if (!d_F[q] || !d_u[q]) return fail(HZ_EINVAL, "null vector");
  hz_problem* pr0 = probs[0];
  hz_options opt = pr0->opt;
  if (o) {
    opt.restart = o->restart;
    opt.maxit = o->maxit;
    opt.tol = o->tol;
    opt.prec = o->prec;
  }
  std::string why;
  if (!valid_options(opt, why)) return fail(HZ_EINVAL, why);
  std::vector<std::unique_ptr<BusyGuard>> guards;
  for (int i = 0; i < nprob; ++i) {
    guards.emplace_back(new BusyGuard(probs[i]->busy));
    if (!guards.back()->ok) return fail(HZ_EBUSY, "problem is in use");
    if (opt.restart > probs[i]->m) return fail(HZ_EINVAL, "restart exceeds the capacity given at creation");
    if (opt.prec == HZ_FP64 && !probs[i]->S)
      return fail(HZ_EINVAL, "problem was created for mixed precision only");
  }
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  try {
    for (int i = 0; i < nprob; ++i)
      if (opt.prec == HZ_MIXED) ensure_mixed_work(probs[i], st);
    const long N = pr0->N;
    std::unique_ptr<Workspace> ws =
        make_workspace(int(nsol), opt.restart, opt.prec, N, pr0->Nc, pr0->G, int(nsol), true);
    std::vector<long> off(nsol);
    for (long q = 0; q < nsol; ++q) {
      off[q] = q * N;
      HZ_HIP(hipMemcpyAsync(ws->Fs + q * N, d_F[q], size_t(N) * 16, hipMemcpyDeviceToDevice, st));
    }
    const hz_status r = lockstep(probs, nprob, nrhs_per_prob, ws->Fs, off.data(), ws->Us,
                                 off.data(), *ws, opt, res, nullptr, st);
    if (r != HZ_OK) return r;
    for (long q = 0; q < nsol; ++q)
      HZ_HIP(hipMemcpyAsync(d_u[q], ws->Us + q * N, size_t(N) * 16, hipMemcpyDeviceToDevice, st));
    HZ_HIP(hipStreamSynchronize(st));
    return HZ_OK;
  } catch (...) {
    return map_exception();
  }
}

size_t hz_batch_workspace_bytes(double h, int p, int nprob, int nrhs_per_prob, const hz_options* o) {
  hz_options d;
  hz_default_options(&d);
  const hz_options& oo = o ? *o : d;
  int n = 0;
  std::string why;
  if (!valid_problem(1.0, h, p, cd(1, 1), n, why) || !valid_options(oo, why) || nprob < 1 ||
      nrhs_per_prob < 1)
    return 0;
  const Sizes z = sizes_of(n, p);
  const int nsol = nprob * nrhs_per_prob;
  return workspace_bytes(z.N, z.nblk, nsol, oo.restart, oo.prec, true) +
         scratch_bytes(z.N, z.Nc, z.G, nsol, oo.prec);
}

hz_status hz_problem_stats(hz_problem* pr, hz_stats* out, int reset) {
  if (!pr || !out) return fail(HZ_EINVAL, "null argument");
  BusyGuard guard(pr->busy);
  if (!guard.ok) return fail(HZ_EBUSY, "problem is in use");
  try {
    collect_timing(pr, true);
    *out = pr->stats;
    if (reset) {
      const double f = pr->stats.factor_ms, ff = pr->stats.factor_flop;
      pr->stats = hz_stats{};
      pr->stats.factor_ms = f;
      pr->stats.factor_flop = ff;
    }
    return HZ_OK;
  } catch (...) {
    return map_exception();
  }
}

void hz_destroy_problem(hz_problem* pr) { delete pr; }

}  // extern "C"

// =========================================================================================
// Serving engine: continuous batching of independent solves
// =========================================================================================

namespace {

struct EnginePool;

struct EngineRequest {
  long id = 0;
  double k = 0, h = 0, theta = 0;
  int p = 1, n = 0;
  cd s;
  const double2* F = nullptr;     // caller's right-hand side, or null: plane-wave load
  double2* u = nullptr;           // caller's solution buffer
  clk::time_point t_submit, t_admit;
  size_t bytes_setup = 0, bytes = 0;
  size_t release_bytes = 0;       // credited to the budget once the reaper has freed them
  hz_problem* pr = nullptr;
  EnginePool* pool = nullptr;
  int slot = -1;
  hz_status status = HZ_OK;
  std::string err;
  bool admitted = false, setup_done = false;
  ~EngineRequest() {
    if (pr) hz_destroy_problem(pr);
  }
};

// A lockstep group of one mesh class (n, p): a workspace of cap solve slots (right-hand
// sides and solutions staged in it) whose members join and leave between rounds.
struct EnginePool {
  int n = 0, p = 0, cap = 0;
  size_t bytes = 0;
  std::unique_ptr<Workspace> ws;
  std::vector<hz_problem*> probs;
  std::vector<EngineRequest*> member;
  std::vector<long> off;
  std::unique_ptr<Lockstep> ls;
  int members() const {
    int c = 0;
    for (auto* r : member) c += r != nullptr;
    return c;
  }
};

struct ClassKey {
  int n, p;
  bool operator<(const ClassKey& o) const { return n != o.n ? n < o.n : p < o.p; }
};
struct ClassState {
  int slots_total = 0;     // slots of created pools plus reserved pools
  int slots_used = 0;      // admitted requests of the class not yet retired
  int reserved = 0;        // pools reserved at admission and not created yet
};

size_t slot_bytes(int n, int p, int m, int prec) {
  const Sizes z = sizes_of(n, p);
  return workspace_bytes(z.N, z.nblk, 1, m, prec, true) + scratch_bytes(z.N, z.Nc, z.G, 1, prec);
}

// Slots per pool: as many solves of the class as fit in about 8 GB of workspace (and a
// quarter of the engine's budget), 1 .. 16.
int pool_cap(int n, int p, int m, int prec, size_t budget) {
  const double b = double(slot_bytes(n, p, m, prec));
  const double lim = std::min(8e9, 0.25 * double(budget));
  return int(std::max(1.0, std::min(16.0, std::floor(lim / b))));
}

size_t request_bytes(int n, int p, int prec, size_t* setup) {
  const Sizes z = sizes_of(n, p);
  // factor, stencil tables, the problem's own one-solve V-cycle scratch and sweep buffer
  const size_t steady = z.factor_elems * (prec == HZ_MIXED ? 8 : 16) +
                        scratch_bytes(z.N, z.Nc, z.G, 1, prec) + 4 * size_t(z.G) * 16 +
                        z.sym_bytes + 256 * 1024;
  // a mixed problem holds the FP64 factor and its FP32 copy while it is set up
  *setup = steady + (prec == HZ_MIXED ? z.factor_elems * 16 : 0);
  return steady;
}

}  // namespace

struct hz_engine {
  hz_engine_config cfg{};
  hz_options opt{};
  int device = 0;
  hipStream_t st_solve = nullptr;
  std::vector<hipStream_t> st_setup;
  std::mutex mu;
  std::condition_variable cv_work, cv_setup, cv_done, cv_trash;
  std::deque<EngineRequest*> pending, setup_q, ready, trash;
  std::deque<std::unique_ptr<EnginePool>> dead_pools;
  std::vector<std::unique_ptr<EnginePool>> pools;   // owned by the loop thread
  std::map<ClassKey, ClassState> classes;           // guarded by mu
  std::deque<hz_engine_result> done;
  size_t used = 0;
  int admitted = 0;                     // admitted and not yet retired
  long submitted = 0, completed = 0;
  bool stop = false;
  std::thread loop, reaper;
  std::vector<std::thread> setup;
  ~hz_engine() {
    pools.clear();
    dead_pools.clear();
    for (auto* r : trash) delete r;
    for (auto* r : pending) delete r;
    for (auto* r : setup_q) delete r;
    for (auto* r : ready) delete r;
    if (st_solve) (void)hipStreamDestroy(st_solve);
    for (auto s : st_setup) (void)hipStreamDestroy(s);
  }
};

namespace {

// Releases the memory of a retired request (and pool slots it reserved); caller holds mu.
// The request's own bytes are credited back by the reaper after the frees have happened:
// a free waits for the device, and the budget must not count memory that is still held.
void engine_release_locked(hz_engine* e, EngineRequest* r) {
  if (!r->admitted) return;
  const size_t b = r->setup_done ? r->bytes : r->bytes_setup;
  if (r->pr) r->release_bytes = b;
  else e->used -= b;                       // a failed set-up freed its memory already
  e->admitted -= 1;
  ClassState& c = e->classes[ClassKey{r->n, r->p}];
  c.slots_used -= 1;
  // a pool reserved for this class and never created is no longer needed
  const int cap = pool_cap(r->n, r->p, e->opt.restart, e->opt.prec, e->cfg.hbm_budget);
  while (c.reserved > 0 && c.slots_total - cap >= c.slots_used) {
    c.reserved -= 1;
    c.slots_total -= cap;
    e->used -= size_t(cap) * slot_bytes(r->n, r->p, e->opt.restart, e->opt.prec);
  }
}

void engine_finish(hz_engine* e, EngineRequest* r, const hz_result* res) {
  hz_engine_result out{};
  out.id = r->id;
  out.status = r->status;
  if (res) out.result = *res;
  const auto now = clk::now();
  out.queue_s = r->admitted ? std::chrono::duration<double>(r->t_admit - r->t_submit).count() : 0.0;
  out.latency_s = std::chrono::duration<double>(now - r->t_submit).count();
  if (r->status != HZ_OK) std::snprintf(out.message, sizeof(out.message), "%s", r->err.c_str());
  {
    std::lock_guard<std::mutex> g(e->mu);
    engine_release_locked(e, r);
    e->done.push_back(out);
    e->completed += 1;
    // device memory is released by the reaper thread: a free may wait for the device
    e->trash.push_back(r);
  }
  e->cv_trash.notify_one();
  e->cv_done.notify_all();
  e->cv_work.notify_all();
}

void engine_reaper_main(hz_engine* e) {
  (void)hipSetDevice(e->device);
  while (true) {
    EngineRequest* r = nullptr;
    std::unique_ptr<EnginePool> pool;
    {
      std::unique_lock<std::mutex> g(e->mu);
      e->cv_trash.wait(g, [&] { return e->stop || !e->trash.empty() || !e->dead_pools.empty(); });
      if (!e->trash.empty()) {
        r = e->trash.front();
        e->trash.pop_front();
      } else if (!e->dead_pools.empty()) {
        pool = std::move(e->dead_pools.front());
        e->dead_pools.pop_front();
      } else {
        return;
      }
    }
    const size_t freed = (r ? r->release_bytes : 0) + (pool ? pool->bytes : 0);
    delete r;
    pool.reset();
    if (freed) {
      {
        std::lock_guard<std::mutex> g(e->mu);
        e->used -= freed;
      }
      e->cv_work.notify_all();
    }
  }
}

// Setup thread: create the problem (tables, coarse factor) on its own stream, so that
// factorisations overlap the solve rounds of the admitted requests.
void engine_setup_main(hz_engine* e, int tid) {
  (void)hipSetDevice(e->device);
  hipStream_t st = e->st_setup[tid];
  while (true) {
    EngineRequest* r = nullptr;
    {
      std::unique_lock<std::mutex> g(e->mu);
      e->cv_setup.wait(g, [&] { return e->stop || !e->setup_q.empty(); });
      if (e->stop) return;
      r = e->setup_q.front();
      e->setup_q.pop_front();
    }
    hz_options o = e->opt;
    o.timing = 0;
    const hz_status stt =
        hz_create_problem(r->k, r->h, r->p, hz_c64{r->s.real(), r->s.imag()}, &o, st, &r->pr);
    if (stt != HZ_OK) {
      r->status = stt;
      r->err = hz_last_error();
      engine_finish(e, r, nullptr);
      continue;
    }
    {
      std::lock_guard<std::mutex> g(e->mu);
      e->used -= r->bytes_setup - r->bytes;      // transient setup memory returned
      r->setup_done = true;
      e->ready.push_back(r);
    }
    e->cv_work.notify_all();
  }
}

// Admits queued requests in arrival order while a slot and the memory budget allow. The
// memory of a new pool is reserved when the class has no free slot left.
void engine_admit(hz_engine* e) {
  while (!e->pending.empty() && e->admitted < e->cfg.max_active) {
    EngineRequest* r = e->pending.front();
    ClassState& c = e->classes[ClassKey{r->n, r->p}];
    size_t need = r->bytes_setup;
    const int cap = pool_cap(r->n, r->p, e->opt.restart, e->opt.prec, e->cfg.hbm_budget);
    const size_t pool_b = size_t(cap) * slot_bytes(r->n, r->p, e->opt.restart, e->opt.prec);
    const bool new_pool = c.slots_used >= c.slots_total;
    if (new_pool) need += pool_b;
    // over the budget only a lone request is admitted, and only when no freed memory is
    // still on its way back
    if (e->used + need > e->cfg.hbm_budget &&
        (e->admitted > 0 || !e->trash.empty() || !e->dead_pools.empty()))
      break;
    e->pending.pop_front();
    if (new_pool) {
      c.slots_total += cap;
      c.reserved += 1;
      e->used += pool_b;
    }
    c.slots_used += 1;
    r->admitted = true;
    r->t_admit = clk::now();
    e->used += r->bytes_setup;
    e->admitted += 1;
    e->setup_q.push_back(r);
    e->cv_setup.notify_one();
  }
}

// Joins a set-up request to a pool of its class (creating a reserved pool if needed).
void engine_join(hz_engine* e, EngineRequest* r, hipStream_t st) {
  EnginePool* pool = nullptr;
  int slot = -1;
  for (auto& pp : e->pools)
    if (pp->n == r->n && pp->p == r->p)
      for (int q = 0; q < pp->cap && slot < 0; ++q)
        if (!pp->member[q]) {
          pool = pp.get();
          slot = q;
        }
  if (!pool) {
    std::unique_ptr<EnginePool> np(new EnginePool());
    const int cap = pool_cap(r->n, r->p, e->opt.restart, e->opt.prec, e->cfg.hbm_budget);
    np->n = r->n;
    np->p = r->p;
    np->cap = cap;
    np->bytes = size_t(cap) * slot_bytes(r->n, r->p, e->opt.restart, e->opt.prec);
    const hz_problem* pr = r->pr;
    np->ws = make_workspace(cap, e->opt.restart, e->opt.prec, pr->N, pr->Nc, pr->G, cap, true);
    np->probs.assign(cap, nullptr);
    np->member.assign(cap, nullptr);
    np->off.resize(cap);
    for (int q = 0; q < cap; ++q) np->off[q] = long(q) * pr->N;
    np->ls.reset(new Lockstep(np->probs.data(), cap, 1, np->ws->Fs, np->off.data(), np->ws->Us,
                              np->off.data(), *np->ws, e->opt));
    np->ls->init_vacant();
    {
      std::lock_guard<std::mutex> g(e->mu);
      ClassState& c = e->classes[ClassKey{r->n, r->p}];
      c.reserved = std::max(0, c.reserved - 1);
    }
    pool = np.get();
    slot = 0;
    e->pools.push_back(std::move(np));
  }
  hz_problem* pr = r->pr;
  double2* Fq = pool->ws->Fs + size_t(slot) * pr->N;
  if (r->F) HZ_HIP(hipMemcpyAsync(Fq, r->F, size_t(pr->N) * 16, hipMemcpyDeviceToDevice, st));
  else launch_planewave(pr->p, pr->n, pr->k, r->theta, pr->gl_t, pr->gl_w, pr->lag, Fq, st);
  pool->probs[slot] = pr;
  pool->member[slot] = r;
  r->pool = pool;
  r->slot = slot;
  const int qs[1] = {slot};
  const hz_status stt = pool->ls->start_slots(qs, 1, nullptr, st);
  if (stt != HZ_OK) throw std::runtime_error(hz_last_error());
}

void engine_leave(hz_engine* e, EngineRequest* r) {
  EnginePool* pool = r->pool;
  if (!pool) return;
  pool->ls->vacate(r->slot);
  pool->probs[r->slot] = nullptr;
  pool->member[r->slot] = nullptr;
  r->pool = nullptr;
  // an empty pool is released unless an admitted request of its class still needs a slot
  if (pool->members() == 0) {
    std::lock_guard<std::mutex> g(e->mu);
    ClassState& c = e->classes[ClassKey{pool->n, pool->p}];
    // the leaving request still counts in slots_used
    if (c.slots_total - pool->cap >= c.slots_used - 1) {
      c.slots_total -= pool->cap;          // its bytes are credited when the reaper frees it
      for (size_t i = 0; i < e->pools.size(); ++i)
        if (e->pools[i].get() == pool) {
          e->dead_pools.push_back(std::move(e->pools[i]));
          e->pools.erase(e->pools.begin() + i);
          break;
        }
    }
  }
  e->cv_trash.notify_one();
}

void engine_fail(hz_engine* e, EngineRequest* r, hz_status stt, const std::string& msg) {
  r->status = stt;
  r->err = msg;
  engine_leave(e, r);
  engine_finish(e, r, nullptr);
}

// Loop thread: every round performs one FGMRES iteration of each active request, one batch
// of launches per pool (all on one stream: the coarse solves are cooperative launches and
// must not run concurrently with each other), synchronises once, then updates every request
// on the host; finished requests leave their pools and free their memory, new ones join
// between rounds.
void engine_loop_main(hz_engine* e) {
  (void)hipSetDevice(e->device);
  hipStream_t st = e->st_solve;
  std::vector<EngineRequest*> joining, finished;
  while (true) {
    bool any = false;
    for (auto& pp : e->pools) any = any || pp->members() > 0;
    {
      std::unique_lock<std::mutex> g(e->mu);
      engine_admit(e);
      if (!any)
        e->cv_work.wait(g, [&] {
          engine_admit(e);
          return e->stop || !e->ready.empty();
        });
      if (e->stop) return;
      joining.assign(e->ready.begin(), e->ready.end());
      e->ready.clear();
    }
    for (EngineRequest* r : joining) {
      try {
        engine_join(e, r, st);
      } catch (...) {
        const hz_status stt = map_exception();
        engine_fail(e, r, stt, hz_last_error());
      }
    }
    joining.clear();
    // one round
    bool issued = false;
    try {
      for (auto& pp : e->pools)
        if (pp->members() > 0) issued = pp->ls->issue(st) || issued;
      HZ_HIP(hipStreamSynchronize(st));
    } catch (...) {
      const hz_status stt = map_exception();
      const std::string msg = hz_last_error();
      std::vector<EngineRequest*> all;
      for (auto& pp : e->pools)
        for (auto* r : pp->member)
          if (r) all.push_back(r);
      for (auto* r : all) engine_fail(e, r, stt, msg);   // may release pools
      continue;
    }
    // host updates; finished solves copy their staged solution out
    finished.clear();
    std::vector<std::pair<EngineRequest*, std::pair<hz_status, std::string>>> failed;
    for (size_t i = 0; i < e->pools.size(); ++i) {
      EnginePool* pp = e->pools[i].get();
      if (pp->members() == 0) continue;
      hz_status stt;
      try {
        stt = pp->ls->complete(st);
      } catch (...) {
        stt = map_exception();
      }
      if (stt != HZ_OK) {
        const std::string msg = hz_last_error();
        for (auto* r : pp->member)
          if (r) failed.push_back({r, {stt, msg}});
        continue;
      }
      for (int q = 0; q < pp->cap; ++q) {
        EngineRequest* r = pp->member[q];
        if (r && pp->ls->S[q].done) {
          if (r->u)
            HZ_HIP(hipMemcpyAsync(r->u, pp->ws->Us + size_t(q) * pp->ws->N,
                                  size_t(pp->ws->N) * 16, hipMemcpyDeviceToDevice, st));
          finished.push_back(r);
        }
      }
    }
    for (auto& f : failed) engine_fail(e, f.first, f.second.first, f.second.second);
    if (finished.empty()) continue;
    try {
      HZ_HIP(hipStreamSynchronize(st));
    } catch (...) {
      const hz_status stt = map_exception();
      for (auto* r : finished) engine_fail(e, r, stt, hz_last_error());
      continue;
    }
    for (EngineRequest* r : finished) {
      EnginePool* pp = r->pool;
      hz_status stt = HZ_OK;
      std::string msg;
      {
        int ef = 0;
        if (hipMemcpy(&ef, r->pr->cw.err, sizeof(int), hipMemcpyDeviceToHost) != hipSuccess || ef) {
          stt = HZ_EDEVICE;
          msg = "coarse solve: a wait for another workgroup timed out";
        }
      }
      if (stt != HZ_OK) {
        engine_fail(e, r, stt, msg);
        continue;
      }
      const hz_result res = pp->ls->result_of(r->slot);
      engine_leave(e, r);
      engine_finish(e, r, &res);
    }
  }
}

}  // namespace

extern "C" {

hz_status hz_engine_default_config(hz_engine_config* c) {
  if (!c) return fail(HZ_EINVAL, "null config");
  c->hbm_budget = 0;
  c->max_active = 64;
  c->setup_threads = 2;
  return HZ_OK;
}

hz_status hz_engine_create(const hz_engine_config* c, const hz_options* o, hz_engine** out) {
  if (!out) return fail(HZ_EINVAL, "null output pointer");
  *out = nullptr;
  hz_engine_config cfg;
  hz_engine_default_config(&cfg);
  if (c) cfg = *c;
  hz_options opt;
  hz_default_options(&opt);
  if (o) opt = *o;
  std::string why;
  if (!valid_options(opt, why)) return fail(HZ_EINVAL, why);
  if (cfg.max_active < 1 || cfg.max_active > 1024) return fail(HZ_EINVAL, "max_active must be in [1, 1024]");
  if (cfg.setup_threads < 1 || cfg.setup_threads > 8) return fail(HZ_EINVAL, "setup_threads must be in [1, 8]");
  hz_engine* e = nullptr;
  try {
    e = new hz_engine();
    e->opt = opt;
    e->opt.timing = 0;
    HZ_HIP(hipGetDevice(&e->device));
    if (cfg.hbm_budget == 0) {
      size_t fr = 0, tot = 0;
      HZ_HIP(hipMemGetInfo(&fr, &tot));
      cfg.hbm_budget = size_t(0.85 * double(fr));
    }
    e->cfg = cfg;
    HZ_HIP(hipStreamCreateWithFlags(&e->st_solve, hipStreamNonBlocking));
    e->st_setup.resize(cfg.setup_threads);
    for (auto& s : e->st_setup) HZ_HIP(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
    e->loop = std::thread(engine_loop_main, e);
    e->reaper = std::thread(engine_reaper_main, e);
    for (int i = 0; i < cfg.setup_threads; ++i) e->setup.emplace_back(engine_setup_main, e, i);
    *out = e;
    return HZ_OK;
  } catch (...) {
    const hz_status stt = map_exception();
    if (e) hz_engine_destroy(e);
    return stt;
  }
}

hz_status hz_engine_submit(hz_engine* e, double k, double h, int p, hz_c64 s, double theta,
                           const hz_c64* d_F, hz_c64* d_u, long req_id) {
  if (!e) return fail(HZ_EINVAL, "null engine");
  int n = 0;
  std::string why;
  const cd sc(s.re, s.im);
  if (!valid_problem(k, h, p, sc, n, why)) return fail(HZ_EINVAL, why);
  if (!d_F && !std::isfinite(theta)) return fail(HZ_EINVAL, "theta must be finite");
  std::unique_ptr<EngineRequest> r(new EngineRequest());
  r->id = req_id;
  r->k = k; r->h = h; r->p = p; r->n = n; r->s = sc; r->theta = theta;
  r->F = reinterpret_cast<const double2*>(d_F);
  r->u = reinterpret_cast<double2*>(d_u);
  r->bytes = request_bytes(n, p, e->opt.prec, &r->bytes_setup);
  const int cap = pool_cap(n, p, e->opt.restart, e->opt.prec, e->cfg.hbm_budget);
  if (r->bytes_setup + size_t(cap) * slot_bytes(n, p, e->opt.restart, e->opt.prec) > e->cfg.hbm_budget)
    return fail(HZ_ENOMEM, "request needs more device memory than the engine budget");
  r->t_submit = clk::now();
  {
    std::lock_guard<std::mutex> g(e->mu);
    if (e->stop) return fail(HZ_EBUSY, "engine is shutting down");
    e->pending.push_back(r.release());
    e->submitted += 1;
  }
  e->cv_work.notify_all();
  return HZ_OK;
}

hz_status hz_engine_poll(hz_engine* e, hz_engine_result* out, int max, int* ndone, int wait_ms) {
  if (!e || !ndone || (max > 0 && !out)) return fail(HZ_EINVAL, "null argument");
  std::unique_lock<std::mutex> g(e->mu);
  if (e->done.empty() && wait_ms > 0)
    e->cv_done.wait_for(g, std::chrono::milliseconds(wait_ms), [&] { return !e->done.empty(); });
  int k = 0;
  while (k < max && !e->done.empty()) {
    out[k++] = e->done.front();
    e->done.pop_front();
  }
  *ndone = k;
  return HZ_OK;
}

hz_status hz_engine_info(hz_engine* e, hz_engine_info_t* info) {
  if (!e || !info) return fail(HZ_EINVAL, "null argument");
  std::lock_guard<std::mutex> g(e->mu);
  info->queued = int(e->pending.size());
  info->admitted = e->admitted;
  info->bytes_in_use = e->used;
  info->hbm_budget = e->cfg.hbm_budget;
  info->submitted = e->submitted;
  info->completed = e->completed;
  return HZ_OK;
}

void hz_engine_destroy(hz_engine* e) {
  if (!e) return;
  {
    std::lock_guard<std::mutex> g(e->mu);
    e->stop = true;
  }
  e->cv_work.notify_all();
  e->cv_setup.notify_all();
  e->cv_trash.notify_all();
  if (e->loop.joinable()) e->loop.join();
  for (auto& t : e->setup)
    if (t.joinable()) t.join();
  if (e->reaper.joinable()) e->reaper.join();
  if (e->st_solve) (void)hipStreamSynchronize(e->st_solve);
  for (auto s : e->st_setup) (void)hipStreamSynchronize(s);
  // requests still in pools
  for (auto& pp : e->pools)
    for (auto*& r : pp->member)
      if (r) {
        delete r;
        r = nullptr;
      }
  delete e;
}

}  // extern "C"

// -----------------------------------------------------------------------------------------
// Shift search (Sec. 5, data generation): for every sample (k, h, p) and its right-hand side,
// the exponent sigma in [sigma_lo, sigma_hi] of the shift eps = k^sigma that minimises the
// average residual reduction rho = (r_end / r_0)^(1 / end) of an FGMRES solve, found by
// golden-section search down to a bracket of width tol. All searches advance concurrently on
// one serving engine: each evaluation is an engine request (set up and factored with its
// shift, solved by continuous batching with the other samples' evaluations).
// -----------------------------------------------------------------------------------------

namespace {

struct SearchState {
  double a = 0, b = 0, c = 0, d = 0, fc = 0, fd = 0;
  bool hc = false, hd = false, done = false;
  int evals = 0;
  double best_rho = 0, best_sigma = 0;
  hz_status status = HZ_OK;
  std::string err;
};

constexpr double kGolden = 0.6180339887498949;   // (sqrt(5) - 1) / 2

// Objective of one solve: (r_end / r_0)^(1 / end); 0 when no iteration was needed.
double search_rho(const hz_result& r) {
  if (r.iterations <= 0) return 0.0;
  return std::pow(r.rel_res_true, 1.0 / r.iterations);
}

}  // namespace

extern "C" {

hz_status hz_shift_search(const hz_search_sample* samples, int n, const hz_c64* const* d_F,
                          double sigma_lo, double sigma_hi, double tol,
                          const hz_engine_config* cfg, const hz_options* o,
                          hz_search_result* out) {
  if (!samples || n < 1 || !d_F || !out) return fail(HZ_EINVAL, "null argument");
  if (!(sigma_lo < sigma_hi) || !std::isfinite(sigma_lo) || !std::isfinite(sigma_hi) ||
      !(tol > 0))
    return fail(HZ_EINVAL, "need sigma_lo < sigma_hi and tol > 0");
  for (int i = 0; i < n; ++i) {
    int nn = 0;
    std::string why;
    if (!d_F[i]) return fail(HZ_EINVAL, "null right-hand side");
    if (!valid_problem(samples[i].k, samples[i].h, samples[i].p, cd(1, 1), nn, why))
      return fail(HZ_EINVAL, "sample " + std::to_string(i) + ": " + why);
  }
  hz_engine* e = nullptr;
  hz_status st = hz_engine_create(cfg, o, &e);
  if (st != HZ_OK) return st;
  std::vector<SearchState> S(n);
  int remaining = n;
  // request id = 2 sample + slot (slot 0: the point c, slot 1: the point d)
  auto submit = [&](int i, int slot) {
    const double sigma = slot == 0 ? S[i].c : S[i].d;
    const double k = samples[i].k;
    const hz_c64 sh{1.0, std::pow(k, sigma - 2.0)};   // eps = k^sigma = Im(s) k^2
    const hz_status r = hz_engine_submit(e, k, samples[i].h, samples[i].p, sh, 0.0, d_F[i],
                                         nullptr, 2L * i + slot);
    if (r != HZ_OK) {
      S[i].status = r;
      S[i].err = hz_last_error();
      S[i].done = true;
      --remaining;
    }
  };
  // advance sample i while both inner points are known
  auto advance = [&](int i) {
    SearchState& z = S[i];
    while (!z.done && z.hc && z.hd) {
      if (z.b - z.a <= tol) {
        z.done = true;
        --remaining;
        break;
      }
      if (z.fc < z.fd) {           // the minimum lies in [a, d]
        z.b = z.d;
        z.d = z.c;
        z.fd = z.fc;
        z.c = z.b - kGolden * (z.b - z.a);
        z.hc = false;
        submit(i, 0);
      } else {                     // in [c, b]
        z.a = z.c;
        z.c = z.d;
        z.fc = z.fd;
        z.d = z.a + kGolden * (z.b - z.a);
        z.hd = false;
        submit(i, 1);
      }
    }
  };
  for (int i = 0; i < n; ++i) {
    SearchState& z = S[i];
    z.a = sigma_lo;
    z.b = sigma_hi;
    z.c = z.b - kGolden * (z.b - z.a);
    z.d = z.a + kGolden * (z.b - z.a);
    z.best_rho = std::numeric_limits<double>::infinity();
    submit(i, 0);
    if (!z.done) submit(i, 1);
  }
  std::vector<hz_engine_result> buf(64);
  while (remaining > 0 && st == HZ_OK) {
    int nd = 0;
    st = hz_engine_poll(e, buf.data(), int(buf.size()), &nd, 200);
    for (int q = 0; q < nd && st == HZ_OK; ++q) {
      const hz_engine_result& r = buf[q];
      const int i = int(r.id / 2), slot = int(r.id % 2);
      SearchState& z = S[i];
      if (z.done) continue;
      if (r.status != HZ_OK) {
        z.status = hz_status(r.status);
        z.err = r.message;
        z.done = true;
        --remaining;
        continue;
      }
      const double rho = search_rho(r.result);
      const double sigma = slot == 0 ? z.c : z.d;
      ++z.evals;
      if (rho < z.best_rho) {
        z.best_rho = rho;
        z.best_sigma = sigma;
      }
      if (slot == 0) { z.fc = rho; z.hc = true; } else { z.fd = rho; z.hd = true; }
      advance(i);
    }
  }
  hz_engine_destroy(e);
  if (st != HZ_OK) return st;
  for (int i = 0; i < n; ++i) {
    out[i].sigma = 0.5 * (S[i].a + S[i].b);
    out[i].rho = S[i].best_rho;
    out[i].sigma_best = S[i].best_sigma;
    out[i].evaluations = S[i].evals;
    out[i].status = S[i].status;
  }
  for (int i = 0; i < n; ++i)
    if (S[i].status != HZ_OK) return fail(S[i].status, "sample " + std::to_string(i) + ": " + S[i].err);
  return HZ_OK;
}

}  // extern "C"
