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
#include <cstdlib>
#include <cstring>
#include <new>

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
  ~DevMem() {
    for (auto& a : live) (void)hipFree(a.first);
  }
};

template <typename T> struct Level {
  DevOp<T> fine, coarse;   // A_eps on the fine and coarse lattices
  const T* rw = nullptr;   // prolongation weights
  const V2<T>* S = nullptr;
  CoarseSolveWork cw;
  V2<T>*ua = nullptr, *ub = nullptr, *rf = nullptr, *rc = nullptr, *ec = nullptr;
};

}  // namespace hz

using namespace hz;

struct hz_problem {
  double k = 0;
  int n = 0, p = 1;
  cd s;
  hz_options opt{};
  int M = 0, Mc = 0;
  long N = 0, Nc = 0;
  CoarseLayout L;
  DevMem mem;
  // FP64 operators and tables
  double2 *cA0 = nullptr, *cAe = nullptr, *wdAe = nullptr, *cAc = nullptr;
  double* rw = nullptr;
  double2* S = nullptr;
  // FP32 operators and tables
  float2 *fcAe = nullptr, *fwdAe = nullptr, *fcAc = nullptr;
  float* frw = nullptr;
  float2* Sf = nullptr;
  // Krylov workspace (restart capacity m)
  int m = 0;
  int nblk = 0;
  double2 *V = nullptr, *Zd = nullptr, *w = nullptr, *r = nullptr, *partial = nullptr,
          *hbuf = nullptr, *ybuf = nullptr;
  double2 *ua = nullptr, *ub = nullptr, *rf = nullptr, *rc = nullptr, *ec = nullptr;
  float2 *Zf = nullptr, *fa = nullptr, *fb = nullptr, *frf = nullptr, *ff = nullptr,
         *frc = nullptr, *fec = nullptr;
  double2* pin = nullptr;   // pinned host read-back buffer
  CoarseSolveWork cw;       // grid-barrier counter and error flag of the coarse solve
  double gl_t[10], gl_w[10], lag[40];
  double setup_s = 0;
  std::atomic<int> busy{0};
  // device-time counters (timing mode): event pairs around each coarse-solve launch
  bool timing = false;
  hz_stats stats{};
  std::vector<std::pair<hipEvent_t, hipEvent_t>> ev_free, ev_pending;
  ~hz_problem() {
    if (pin) (void)hipHostFree(pin);
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

struct Sizes {
  long N, Nc;
  size_t factor_elems, maxblock;
  int nblk;
};
Sizes sizes_of(int n, int p) {
  Sizes z;
  const int M = p * n + 1, Mc = p * (n / 2) + 1;
  z.N = long(M) * M;
  z.Nc = long(Mc) * Mc;
  CoarseLayout L{p, n / 2, Mc};
  z.factor_elems = L.total();
  z.maxblock = size_t(L.size(0));
  z.nblk = mdot_blocks(z.N);
  return z;
}

// Device bytes of the resident parts (factor, tables, workspace) for a precision.
size_t resident_bytes(int n, int p, int m, int prec) {
  const Sizes z = sizes_of(n, p);
  size_t b = 0;
  b += z.factor_elems * (prec == HZ_MIXED ? 8 : 16);
  b += size_t(m + 1) * z.N * 16;                       // V
  b += size_t(m) * z.N * (prec == HZ_MIXED ? 8 : 16);  // Z
  b += 2 * size_t(z.N) * 16;                           // w, r
  if (prec == HZ_MIXED) b += 4 * size_t(z.N) * 8 + 2 * size_t(z.Nc) * 8;
  else b += 3 * size_t(z.N) * 16 + 2 * size_t(z.Nc) * 16;
  b += size_t(z.nblk) * 64 * 16 + 4096 + 64 * 1024;   // partials, small buffers, tables
  return b;
}

void upload_tables(hz_problem* pr) {
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
    HZ_HIP(hipMemcpy(d, v.data(), v.size() * 16, hipMemcpyHostToDevice));
    if (want_f) {
      std::vector<float2> fv(v.size());
      for (size_t i = 0; i < v.size(); ++i) fv[i] = make_float2(float(v[i].real()), float(v[i].imag()));
      f = pr->mem.alloc<float2>(v.size());
      HZ_HIP(hipMemcpy(f, fv.data(), v.size() * 8, hipMemcpyHostToDevice));
    }
  };
  float2* dummy = nullptr;
  up2(a0, pr->cA0, dummy, false);
  up2(ae, pr->cAe, pr->fcAe, true);
  up2(wd, pr->wdAe, pr->fwdAe, true);
  up2(ac, pr->cAc, pr->fcAc, true);
  pr->rw = pr->mem.alloc<double>(ft.RW.size());
  HZ_HIP(hipMemcpy(pr->rw, ft.RW.data(), ft.RW.size() * 8, hipMemcpyHostToDevice));
  std::vector<float> frw(ft.RW.begin(), ft.RW.end());
  pr->frw = pr->mem.alloc<float>(frw.size());
  HZ_HIP(hipMemcpy(pr->frw, frw.data(), frw.size() * 4, hipMemcpyHostToDevice));
  gauss_legendre10(pr->gl_t, pr->gl_w);
  for (int l = 0; l < 4; ++l)
    for (int q = 0; q < 10; ++q) {
      double v = 1.0;
      for (int mm = 0; mm <= p; ++mm)
        if (mm != l) v *= (pr->gl_t[q] - double(mm) / p) / (double(l) / p - double(mm) / p);
      pr->lag[l * 10 + q] = (l <= p) ? v : 0.0;
    }
}

void ensure_fp64_work(hz_problem* pr) {
  if (pr->Zd) return;
  pr->Zd = pr->mem.alloc<double2>(size_t(pr->m) * pr->N);
  pr->ua = pr->mem.alloc<double2>(pr->N);
  pr->ub = pr->mem.alloc<double2>(pr->N);
  pr->rf = pr->mem.alloc<double2>(pr->N);
  pr->rc = pr->mem.alloc<double2>(pr->Nc);
  pr->ec = pr->mem.alloc<double2>(pr->Nc);
}

void ensure_mixed_work(hz_problem* pr, hipStream_t st) {
  if (!pr->Sf) {
    pr->Sf = pr->mem.alloc<float2>(pr->L.total());
    launch_factor_to_f32(pr->S, pr->Sf, pr->L.total(), st);
  }
  if (pr->Zf) return;
  pr->Zf = pr->mem.alloc<float2>(size_t(pr->m) * pr->N);
  pr->fa = pr->mem.alloc<float2>(pr->N);
  pr->fb = pr->mem.alloc<float2>(pr->N);
  pr->frf = pr->mem.alloc<float2>(pr->N);
  pr->ff = pr->mem.alloc<float2>(pr->N);
  pr->frc = pr->mem.alloc<float2>(pr->Nc);
  pr->fec = pr->mem.alloc<float2>(pr->Nc);
}

Level<double> level64(hz_problem* pr) {
  Level<double> l;
  l.fine = DevOp<double>{pr->cAe, pr->wdAe, pr->M};
  l.coarse = DevOp<double>{pr->cAc, nullptr, pr->Mc};
  l.rw = pr->rw;
  l.S = pr->S;
  l.cw = pr->cw;
  l.ua = pr->ua; l.ub = pr->ub; l.rf = pr->rf; l.rc = pr->rc; l.ec = pr->ec;
  return l;
}
Level<float> level32(hz_problem* pr) {
  Level<float> l;
  l.fine = DevOp<float>{pr->fcAe, pr->fwdAe, pr->M};
  l.coarse = DevOp<float>{pr->fcAc, nullptr, pr->Mc};
  l.rw = pr->frw;
  l.S = pr->Sf;
  l.cw = pr->cw;
  l.ua = pr->fa; l.ub = pr->fb; l.rf = pr->frf; l.rc = pr->frc; l.ec = pr->fec;
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

template <typename T>
void timed_coarse_solve(hz_problem* pr, const Level<T>& lv, const V2<T>* S, const V2<T>* b,
                        V2<T>* y, hipStream_t st) {
  pr->stats.coarse_solves += 1;
  if (!pr->timing) {
    coarse_solve<T>(pr->L, lv.coarse, S, b, y, 1, 0, lv.cw, st);
    return;
  }
  auto e = take_events(pr);
  HZ_HIP(hipEventRecord(e.first, st));
  coarse_solve<T>(pr->L, lv.coarse, S, b, y, 1, 0, lv.cw, st);
  HZ_HIP(hipEventRecord(e.second, st));
  pr->ev_pending.push_back(e);
  if (pr->ev_pending.size() > 64) collect_timing(pr, true);
}

// One twogrid V(nu, nu)-cycle from a zero initial guess (Algorithm 1, two levels):
// nu damped Jacobi sweeps, r_c = P^T (f - A_eps u), e_c = A_c^{-1} r_c, u += P e_c,
// nu sweeps. The last sweep writes z.
template <typename T>
void vcycle(hz_problem* pr, const Level<T>& lv, int nu, const V2<T>* f, V2<T>* z,
            hipStream_t st) {
  pr->stats.vcycles += 1;
  const int p = pr->p;
  V2<T>* cur = lv.ua;
  V2<T>* nxt = lv.ub;
  if (nu == 0) {
    launch_restrict<T>(p, pr->M, pr->Mc, lv.rw, f, lv.rc, 1, 0, 0, st);
    launch_fill_zero(cur, pr->N, st);
  } else {
    launch_jacobi0<T, T>(p, lv.fine, f, cur, 1, 0, st);
    for (int sw = 1; sw < nu; ++sw) {
      launch_stencil<T, T, T, T>(p, ST_SMOOTH, lv.fine, cur, f, nxt, 1, 0, st);
      std::swap(cur, nxt);
    }
    launch_stencil<T, T, T, T>(p, ST_RESID, lv.fine, cur, f, lv.rf, 1, 0, st);
    launch_restrict<T>(p, pr->M, pr->Mc, lv.rw, lv.rf, lv.rc, 1, 0, 0, st);
  }
  timed_coarse_solve<T>(pr, lv, lv.S, lv.rc, lv.ec, st);
  launch_prolong<T>(p, pr->M, pr->Mc, lv.rw, lv.ec, cur, true, 1, 0, 0, st);
  if (nu == 0) {
    HZ_HIP(hipMemcpyAsync(z, cur, sizeof(V2<T>) * pr->N, hipMemcpyDeviceToDevice, st));
    return;
  }
  for (int sw = 0; sw < nu; ++sw) {
    V2<T>* dst = (sw == nu - 1) ? z : nxt;
    launch_stencil<T, T, T, T>(p, ST_SMOOTH, lv.fine, cur, f, dst, 1, 0, st);
    nxt = cur;
    cur = dst;
  }
}

// ||x||_2 of a fine vector through the fixed-order reduction (synchronises).
double norm2(hz_problem* pr, const double2* x, hipStream_t st) {
  launch_mdot<double>(x, 0, 1, x, pr->N, pr->partial, pr->nblk, st);
  launch_reduce(pr->partial, pr->nblk, 1, pr->hbuf, st);
  HZ_HIP(hipMemcpyAsync(pr->pin, pr->hbuf, 16, hipMemcpyDeviceToHost, st));
  HZ_HIP(hipStreamSynchronize(st));
  return std::sqrt(pr->pin[0].x);
}

void precondition(hz_problem* pr, bool mixed, const double2* v, int j, hipStream_t st) {
  if (!mixed) {
    vcycle<double>(pr, level64(pr), pr->opt.nu, v, pr->Zd + size_t(j) * pr->N, st);
  } else {
    launch_d2f(v, pr->ff, pr->N, st);
    vcycle<float>(pr, level32(pr), pr->opt.nu, pr->ff, pr->Zf + size_t(j) * pr->N, st);
  }
}

void apply_A0_z(hz_problem* pr, bool mixed, int j, double2* out, hipStream_t st) {
  const DevOp<double> a0{pr->cA0, nullptr, pr->M};
  if (!mixed)
    launch_stencil<double, double, double, double>(pr->p, ST_APPLY, a0, pr->Zd + size_t(j) * pr->N,
                                                   nullptr, out, 1, 0, st);
  else
    launch_stencil<double, float, double, double>(pr->p, ST_APPLY, a0, pr->Zf + size_t(j) * pr->N,
                                                  nullptr, out, 1, 0, st);
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

hz_status solve_impl(hz_problem* pr, const double2* F, double2* u, const hz_options& o,
                     hz_result* res, double* hist, hipStream_t st) {
  const auto t0 = clk::now();
  const bool mixed = o.prec == HZ_MIXED;
  if (o.restart > pr->m) return fail(HZ_EINVAL, "restart exceeds the capacity given at creation");
  if (mixed) ensure_mixed_work(pr, st);
  else {
    if (!pr->S) return fail(HZ_EINVAL, "problem was created for mixed precision only");
    ensure_fp64_work(pr);
  }
  const long N = pr->N;
  const int m = o.restart;
  const double normF = norm2(pr, F, st);
  if (!std::isfinite(normF)) return fail(HZ_EINVAL, "right-hand side is not finite");
  launch_fill_zero(u, N, st);
  hz_result out{};
  out.setup_s = pr->setup_s;
  out.converged = 1;
  if (normF == 0.0) {
    HZ_HIP(hipStreamSynchronize(st));
    out.solve_s = secs(t0);
    if (res) *res = out;
    return HZ_OK;
  }
  launch_axpby_copy(F, pr->r, N, st);
  double beta = normF;
  int its = 0;
  bool conv = false;
  double true_rel = 1.0, est = 1.0;
  std::vector<cd> H(size_t(m + 1) * m), g(m + 1), y(m);
  std::vector<double> cs(m);
  std::vector<cd> sn(m);
  auto Hat = [&](int i, int j) -> cd& { return H[size_t(i) * m + j]; };
  double2* h1 = pr->hbuf;
  double2* h2 = pr->hbuf + 64;
  double2* hn = pr->hbuf + 128;
  while (true) {
    launch_scale(pr->r, 1.0 / beta, pr->V, N, st);
    std::fill(H.begin(), H.end(), cd(0, 0));
    std::fill(g.begin(), g.end(), cd(0, 0));
    g[0] = beta;
    int jend = 0;
    for (int j = 0; j < m; ++j) {
      const double2* vj = pr->V + size_t(j) * N;
      precondition(pr, mixed, vj, j, st);
      apply_A0_z(pr, mixed, j, pr->w, st);
      ++its;
      // CGS2: two passes of h = V^H w, w -= V h
      launch_mdot<double>(pr->V, N, j + 1, pr->w, N, pr->partial, pr->nblk, st);
      launch_reduce(pr->partial, pr->nblk, j + 1, h1, st);
      launch_maxpy(pr->V, N, j + 1, h1, pr->w, N, nullptr, pr->nblk, st);
      launch_mdot<double>(pr->V, N, j + 1, pr->w, N, pr->partial, pr->nblk, st);
      launch_reduce(pr->partial, pr->nblk, j + 1, h2, st);
      launch_maxpy(pr->V, N, j + 1, h2, pr->w, N, pr->partial, pr->nblk, st);
      launch_reduce(pr->partial, pr->nblk, 1, hn, st);
      HZ_HIP(hipMemcpyAsync(pr->pin, pr->hbuf, 129 * 16, hipMemcpyDeviceToHost, st));
      HZ_HIP(hipStreamSynchronize(st));
      if (pr->timing) collect_timing(pr, false);
      for (int i = 0; i <= j; ++i)
        Hat(i, j) = (cd(0, 0) + cd(pr->pin[i].x, pr->pin[i].y)) + cd(pr->pin[64 + i].x, pr->pin[64 + i].y);
      const double hnext = std::sqrt(pr->pin[128].x);
      if (!std::isfinite(hnext)) return fail(HZ_EDEVICE, "non-finite Arnoldi norm");
      Hat(j + 1, j) = hnext;
      if (hnext > 0) launch_scale(pr->w, 1.0 / hnext, pr->V + size_t(j + 1) * N, N, st);
      for (int i = 0; i < j; ++i) {
        const cd a = Hat(i, j), b = Hat(i + 1, j);
        Hat(i, j) = cs[i] * a + sn[i] * b;
        Hat(i + 1, j) = -std::conj(sn[i]) * a + cs[i] * b;
      }
      givens(Hat(j, j), Hat(j + 1, j), cs[j], sn[j]);
      {
        const cd a = Hat(j, j), b = Hat(j + 1, j);
        Hat(j, j) = cs[j] * a + sn[j] * b;
        Hat(j + 1, j) = 0;
      }
      g[j + 1] = -std::conj(sn[j]) * g[j];
      g[j] = cs[j] * g[j];
      est = std::abs(g[j + 1]) / normF;
      if (hist) hist[its - 1] = est;
      jend = j + 1;
      if (est <= o.tol || its >= o.maxit || hnext == 0.0) break;
    }
    for (int i = jend - 1; i >= 0; --i) {
      cd acc = g[i];
      for (int l = i + 1; l < jend; ++l) acc -= Hat(i, l) * y[l];
      y[i] = acc / Hat(i, i);
    }
    HZ_HIP(hipMemcpyAsync(pr->ybuf, y.data(), size_t(jend) * 16, hipMemcpyHostToDevice, st));
    if (!mixed) launch_update<double>(pr->Zd, N, jend, pr->ybuf, u, N, st);
    else launch_update<float>(pr->Zf, N, jend, pr->ybuf, u, N, st);
    const DevOp<double> a0{pr->cA0, nullptr, pr->M};
    launch_stencil<double, double, double, double>(pr->p, ST_RESID, a0, u, F, pr->r, 1, 0, st);
    beta = norm2(pr, pr->r, st);   // synchronises: y (host) stays alive until the copy ran
    true_rel = beta / normF;
    if (true_rel <= o.tol) {
      conv = true;
      break;
    }
    if (its >= o.maxit) break;
  }
  {
    int e = 0;
    HZ_HIP(hipMemcpy(&e, pr->cw.err, sizeof(int), hipMemcpyDeviceToHost));
    if (e) return fail(HZ_EDEVICE, "coarse solve grid barrier timed out");
  }
  out.iterations = its;
  out.converged = conv ? 1 : 0;
  out.rel_res_true = true_rel;
  out.rel_res_est = est;
  out.solve_s = secs(t0);
  if (res) *res = out;
  return HZ_OK;
}

}  // namespace

// =========================================================================================
// C ABI
// =========================================================================================

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
    pr->nblk = mdot_blocks(pr->N);
    upload_tables(pr);
    // coarse factor (FP64), then the FP32 copy for mixed-precision problems
    pr->S = pr->mem.alloc<double2>(pr->L.total());
    {
      CoarseFactorWork wk;
      const size_t mb = size_t(pr->L.size(0));
      wk.T = pr->mem.alloc<double2>(2 * mb * mb);     // one set per factorisation chain
      wk.W = pr->mem.alloc<double2>(2 * mb * 32);
      wk.R = pr->mem.alloc<double2>(2 * mb * 32);
      wk.flag = pr->mem.alloc<int>(1);
      const DevOp<double> cop{pr->cAc, nullptr, pr->Mc};
      pr->timing = opt.timing != 0;
      hipEvent_t f0 = nullptr, f1 = nullptr;
      if (pr->timing) {
        HZ_HIP(hipEventCreate(&f0));
        HZ_HIP(hipEventCreate(&f1));
        HZ_HIP(hipEventRecord(f0, st));
      }
      const hz_status fs = coarse_factor(pr->L, cop, pr->S, wk, st);
      if (pr->timing) {
        HZ_HIP(hipEventRecord(f1, st));
        HZ_HIP(hipEventSynchronize(f1));
        float ms = 0;
        HZ_HIP(hipEventElapsedTime(&ms, f0, f1));
        pr->stats.factor_ms = ms;
        (void)hipEventDestroy(f0);
        (void)hipEventDestroy(f1);
      }
      pr->mem.release(wk.T);
      pr->mem.release(wk.W);
      pr->mem.release(wk.R);
      pr->mem.release(wk.flag);
      if (fs != HZ_OK) {
        delete pr;
        return fail(fs, "zero or non-finite pivot in the coarse block factorisation");
      }
    }
    pr->V = pr->mem.alloc<double2>(size_t(pr->m + 1) * pr->N);
    pr->w = pr->mem.alloc<double2>(pr->N);
    pr->r = pr->mem.alloc<double2>(pr->N);
    pr->partial = pr->mem.alloc<double2>(size_t(pr->nblk) * 64);
    pr->hbuf = pr->mem.alloc<double2>(4 * 64);
    pr->ybuf = pr->mem.alloc<double2>(64);
    pr->cw.g = pr->mem.alloc<double2>(4 * size_t(pr->Nc));
    pr->cw.err = pr->mem.alloc<int>(64);
    HZ_HIP(hipMemsetAsync(pr->cw.err, 0, 64 * sizeof(int), st));
    {
      const char* env = std::getenv("HZ_COARSE_PERSISTENT");
      pr->cw.persistent = !(env && env[0] == '0');
    }
    HZ_HIP(hipHostMalloc(reinterpret_cast<void**>(&pr->pin), 4 * 64 * 16, hipHostMallocDefault));
    if (opt.prec == HZ_MIXED) {
      ensure_mixed_work(pr, st);
      HZ_HIP(hipStreamSynchronize(st));
      pr->mem.release(pr->S);
      pr->S = nullptr;
    } else {
      ensure_fp64_work(pr);
    }
    HZ_HIP(hipStreamSynchronize(st));
    pr->setup_s = secs(t0);
    *out = pr;
    return HZ_OK;
  } catch (...) {
    delete pr;
    return map_exception();
  }
}

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
  if (!pr || !d_x || !d_y) return fail(HZ_EINVAL, "null argument");
  if ((op == HZ_OP_JACOBI || op == HZ_OP_RESID_RESTRICT) && !d_f)
    return fail(HZ_EINVAL, "this operator needs d_f");
  if (op < 0 || op > HZ_OP_RESID_RESTRICT) return fail(HZ_EINVAL, "unknown operator");
  if (prec != HZ_FP64 && prec != HZ_MIXED) return fail(HZ_EINVAL, "bad precision");
  BusyGuard guard(pr->busy);
  if (!guard.ok) return fail(HZ_EBUSY, "problem is in use");
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  const double2* x = reinterpret_cast<const double2*>(d_x);
  const double2* f = reinterpret_cast<const double2*>(d_f);
  double2* y = reinterpret_cast<double2*>(d_y);
  const int p = pr->p;
  const bool fine_in = !(op == HZ_OP_PROLONG || op == HZ_OP_COARSE_SOLVE || op == HZ_OP_COARSE_A);
  const bool fine_out = !(op == HZ_OP_RESTRICT || op == HZ_OP_COARSE_SOLVE ||
                          op == HZ_OP_COARSE_A || op == HZ_OP_RESID_RESTRICT);
  try {
    if (prec == HZ_FP64) {
      if (!pr->S) return fail(HZ_EINVAL, "problem was created for mixed precision only");
      ensure_fp64_work(pr);
      const Level<double> lv = level64(pr);
      const DevOp<double> a0{pr->cA0, nullptr, pr->M};
      switch (op) {
        case HZ_OP_A0: launch_stencil<double, double, double, double>(p, ST_APPLY, a0, x, nullptr, y, 1, 0, st); break;
        case HZ_OP_AEPS: launch_stencil<double, double, double, double>(p, ST_APPLY, lv.fine, x, nullptr, y, 1, 0, st); break;
        case HZ_OP_JACOBI: launch_stencil<double, double, double, double>(p, ST_SMOOTH, lv.fine, x, f, y, 1, 0, st); break;
        case HZ_OP_RESTRICT: launch_restrict<double>(p, pr->M, pr->Mc, pr->rw, x, y, 1, 0, 0, st); break;
        case HZ_OP_PROLONG: launch_prolong<double>(p, pr->M, pr->Mc, pr->rw, x, y, false, 1, 0, 0, st); break;
        case HZ_OP_VCYCLE: vcycle<double>(pr, lv, pr->opt.nu, x, y, st); break;
        case HZ_OP_COARSE_SOLVE: timed_coarse_solve<double>(pr, lv, pr->S, x, y, st); break;
        case HZ_OP_COARSE_A: launch_stencil<double, double, double, double>(p, ST_APPLY, lv.coarse, x, nullptr, y, 1, 0, st); break;
        case HZ_OP_RESID_RESTRICT:
          launch_stencil<double, double, double, double>(p, ST_RESID, lv.fine, x, f, pr->rf, 1, 0, st);
          launch_restrict<double>(p, pr->M, pr->Mc, pr->rw, pr->rf, y, 1, 0, 0, st);
          break;
      }
    } else {
      ensure_mixed_work(pr, st);
      const Level<float> lv = level32(pr);
      const long nin = fine_in ? pr->N : pr->Nc;
      const long nout = fine_out ? pr->N : pr->Nc;
      // inputs to FP32 scratch: x -> ff (fine) or frc (coarse); f -> fb
      float2* xin = fine_in ? pr->ff : pr->frc;
      launch_d2f(x, xin, nin, st);
      if (f) launch_d2f(f, pr->fb, pr->N, st);
      float2* yout = fine_out ? pr->frf : pr->fec;
      if (op == HZ_OP_VCYCLE || op == HZ_OP_RESID_RESTRICT) yout = fine_out ? pr->Zf : pr->fec;
      switch (op) {
        case HZ_OP_A0: {
          const DevOp<double> a0{pr->cA0, nullptr, pr->M};
          launch_stencil<double, float, double, double>(p, ST_APPLY, a0, xin, nullptr, y, 1, 0, st);
          return HZ_OK;
        }
        case HZ_OP_AEPS: launch_stencil<float, float, float, float>(p, ST_APPLY, lv.fine, xin, nullptr, yout, 1, 0, st); break;
        case HZ_OP_JACOBI: launch_stencil<float, float, float, float>(p, ST_SMOOTH, lv.fine, xin, pr->fb, yout, 1, 0, st); break;
        case HZ_OP_RESTRICT: launch_restrict<float>(p, pr->M, pr->Mc, pr->frw, xin, yout, 1, 0, 0, st); break;
        case HZ_OP_PROLONG: launch_prolong<float>(p, pr->M, pr->Mc, pr->frw, xin, yout, false, 1, 0, 0, st); break;
        case HZ_OP_VCYCLE: vcycle<float>(pr, lv, pr->opt.nu, xin, yout, st); break;
        case HZ_OP_COARSE_SOLVE: timed_coarse_solve<float>(pr, lv, pr->Sf, xin, yout, st); break;
        case HZ_OP_COARSE_A: launch_stencil<float, float, float, float>(p, ST_APPLY, lv.coarse, xin, nullptr, yout, 1, 0, st); break;
        case HZ_OP_RESID_RESTRICT:
          launch_stencil<float, float, float, float>(p, ST_RESID, lv.fine, xin, pr->fb, pr->frf, 1, 0, st);
          launch_restrict<float>(p, pr->M, pr->Mc, pr->frw, pr->frf, yout, 1, 0, 0, st);
          break;
      }
      launch_f2d(yout, y, nout, st);
    }
    return HZ_OK;
  } catch (...) {
    return map_exception();
  }
}

hz_status hz_solve_batched(hz_problem* const* probs, int nprob, const hz_c64* const* d_F,
                           int nrhs_per_prob, hz_c64* const* d_u, const hz_options* o,
                           hz_result* res, void* hip_stream) {
  if (!probs || nprob < 1 || nrhs_per_prob < 1 || !d_F || !d_u) return fail(HZ_EINVAL, "bad arguments");
  for (int i = 0; i < nprob; ++i) {
    if (!probs[i]) return fail(HZ_EINVAL, "null problem");
    if (probs[i]->n != probs[0]->n || probs[i]->p != probs[0]->p || probs[i]->k != probs[0]->k)
      return fail(HZ_EINVAL, "batched problems must share (k, h, p)");
  }
  for (int i = 0; i < nprob; ++i)
    for (int r = 0; r < nrhs_per_prob; ++r) {
      const int q = i * nrhs_per_prob + r;
      const hz_status stt = hz_solve(probs[i], d_F[q], d_u[q], o, res ? res + q : nullptr, nullptr, hip_stream);
      if (stt != HZ_OK) return stt;
    }
  return HZ_OK;
}

hz_status hz_problem_stats(hz_problem* pr, hz_stats* out, int reset) {
  if (!pr || !out) return fail(HZ_EINVAL, "null argument");
  BusyGuard guard(pr->busy);
  if (!guard.ok) return fail(HZ_EBUSY, "problem is in use");
  try {
    collect_timing(pr, true);
    *out = pr->stats;
    if (reset) {
      const double f = pr->stats.factor_ms;
      pr->stats = hz_stats{};
      pr->stats.factor_ms = f;
    }
    return HZ_OK;
  } catch (...) {
    return map_exception();
  }
}

void hz_destroy_problem(hz_problem* pr) { delete pr; }

}  // extern "C"
