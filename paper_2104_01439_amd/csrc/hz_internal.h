// Internal declarations of the HIP Helmholtz solver (not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <complex>
#include <cstdint>
#include <string>
#include <vector>

#include "hz.h"

namespace hz {

using cd = std::complex<double>;

// ------------------------------------------------------------------------------------------
// Host tables (hz_tables.cpp)
// ------------------------------------------------------------------------------------------

struct RefElement {
  int p, nloc;
  int ni[10], nj[10];     // local node (i, j) sits at (i/p, j/p) of the reference triangle
  int ma[10], mb[10];     // monomials x^ma y^mb
  double C[10][10];       // phi_k = sum_m C[m][k] x^ma[m] y^mb[m]
  explicit RefElement(int p);
  double phi(int k, double x, double y) const;
};

// Stencil tables of one level (fine or coarse), real parts of K, M and the unit-weight
// boundary mass, indexed [cls * 9 + reg][(dy + p) * (2p+1) + (dx + p)], with
// cls = (b mod p) * p + (a mod p) and reg = ry * 3 + rx (0: first line, 1: interior,
// 2: last line of the lattice along that axis). RW holds the prolongation weights
// [cls][(dy + 2p) * (4p+1) + (dx + 2p)] (coarse class, fine offsets).
struct LevelTables {
  int p = 1, n = 0, M = 0;
  double h = 0;
  std::vector<double> K, Mm, B, RW;
};

LevelTables build_level_tables(int p, int n, double h);

// Per-cell coefficient tables of one level whose cells are r x r fine cells (r = 1: the fine
// level, r = 2: the coarse level), fine cell side hf. For a lattice point of class
// cls = (b mod p) p + (a mod p) in level cell (A0, B0) = (a div p, b div p) and a neighbour
// offset d = (dy + p)(2p + 1) + (dx + p), entry f = (fy + r) 2r + (fx + r) holds the integrals
// over fine cell (r A0 + fx, r B0 + fy), fx, fy in [-r, r), of grad phi_i . grad phi_j (K) and
// phi_i phi_j (Mm): K[(cls W2 + d) 4r^2 + f]. B[(cc (2p+1) + (e + p)) 2r + (fe + r)] is the
// integral of the boundary traces over fine boundary edge r E0 + fe of a point at position
// p E0 + cc along a side, neighbour at offset e along the same side.
struct CellTables {
  int p = 1, r = 1;
  std::vector<double> K, Mm, B;
};
CellTables build_cell_tables(int p, int r, double hf);

// Collapsed q x q Gauss-Legendre rule on the reference triangle (xi, eta, w), the basis values
// phi[r * nq + k] and loc[cls * 8 + ((Bc + 1) 2 + (Ac + 1)) 2 + tri]: the local index of a
// point of class cls in triangle tri of the cell at (Ac, Bc) in {-1, 0}^2 from its own, or -1.
struct QuadTables {
  int p = 1, nq = 0;
  std::vector<double> xi, eta, w, phi;
  std::vector<int> loc;
};
QuadTables build_quad_tables(int p, int q);
std::vector<cd> combine_operator(const LevelTables& t, double k, cd s);

// ------------------------------------------------------------------------------------------
// Device-side views
// ------------------------------------------------------------------------------------------

template <typename T> struct vec2;
template <> struct vec2<double> { using type = double2; };
template <> struct vec2<float> { using type = float2; };
template <typename T> using V2 = typename vec2<T>::type;

// Element offset of batch element z of a set of vectors: off[z] when a device table is
// given (gathers from arbitrary places of one allocation), else z * stride.
struct Addr {
  long stride = 0;
  const long* off = nullptr;
  __host__ __device__ Addr() {}
  __host__ __device__ Addr(long s) : stride(s) {}
  __host__ __device__ Addr(long s, const long* o) : stride(s), off(o) {}
  __device__ __forceinline__ long at(int z) const { return off ? off[z] : long(z) * stride; }
};

// One level's operator on the device: complex stencil coefficients and the Jacobi
// multiplier omega / diag(A) per (class, region).
// A batched launch may give every batch element its own operator (problems of one mesh
// class with different k or shift): ctab / wtab are then device tables of per-element
// pointers that replace coef / wdinv.
// With pn = 1 the operator varies from point to point (heterogeneous k): coef holds one
// stencil per lattice point, [(2p+1)^2][M*M] (offset-major), and wdinv one multiplier per
// point, [M*M].
template <typename T> struct DevOp {
  const V2<T>* coef = nullptr;   // [p*p*9][(2p+1)^2]
  const V2<T>* wdinv = nullptr;  // [p*p*9]
  int M = 0;                     // lattice points per side
  const V2<T>* const* ctab = nullptr;
  const V2<T>* const* wtab = nullptr;
  int pn = 0;
};

// Coarse block-tridiagonal factor: block j (j < nc) holds lattice rows p j .. p j + p - 1,
// the last block (j = nc) holds the final lattice row alone. Block j stores the dense
// inverse S_j of the Schur complement D_j, row-major, at element offset off(j).
struct CoarseLayout {
  int p = 1, nc = 0, Mc = 0;     // coarse cells per side, coarse lattice points per side
  int nblocks() const { return nc + 1; }
  int rows(int j) const { return j < nc ? p : 1; }
  long size(int j) const { return long(rows(j)) * Mc; }
  long first_dof(int j) const { return long(p) * j * Mc; }
  size_t off(int j) const { return size_t(j) * size_t(p * Mc) * size_t(p * Mc); }
  size_t total() const { return off(nc) + size_t(Mc) * size_t(Mc); }
};

// ------------------------------------------------------------------------------------------
// Launchers (hz_fine.hip, hz_coarse.hip, hz_krylov.hip)
// ------------------------------------------------------------------------------------------

enum StencilMode { ST_APPLY = 0, ST_RESID = 1, ST_SMOOTH = 2, ST_SMOOTH0 = 3, ST_SMOOTH_PC = 4 };

// y = A x  |  y = f - A x  |  y = x + wdinv (f - A x)   on one level, lattice M x M;
// ST_SMOOTH0: the first two Jacobi sweeps from a zero iterate in one pass, y = u1 + wdinv
// (f - A u1) with u1 = wdinv f formed while staging (x must be f, with the same offsets);
// bitwise the result of the first sweep followed by an ST_SMOOTH sweep.
// nbatch independent vectors, batch element z at x + ax.at(z), f + af.at(z), y + ay.at(z).
template <typename T, typename TX, typename TF, typename TY>
void launch_stencil(int p, int mode, const DevOp<T>& op, const V2<TX>* x, Addr ax,
                    const V2<TF>* f, Addr af, V2<TY>* y, Addr ay, int nbatch, hipStream_t st);
// The first post-smoothing sweep with the coarse-grid correction (Alg. 1): y = v + wdinv
// (f - A v) with v = x + P ec formed while staging (coarse vector ec at ec + ac.at(z), Mc x Mc
// lattice, prolongation weights rw); bitwise the prolongation-add followed by an ST_SMOOTH
// sweep. Returns false (launching nothing) where it is not provided: per-point operators and
// p = 3, whose staged tiles would not leave room for the coarse tile.
template <typename T>
bool launch_smooth_pc(int p, const DevOp<T>& op, const V2<T>* x, Addr ax, const V2<T>* ec,
                      Addr ac, int Mc, const T* rw, const V2<T>* f, Addr af, V2<T>* y, Addr ay,
                      int nbatch, hipStream_t st);
// Residual and restriction in one pass (Alg. 1: restrict residual): yc = P^T (f - A x), fine
// lattice op.M, coarse Mc, batch offsets as for launch_stencil; bitwise the ST_RESID pass
// followed by launch_restrict. Returns false (launching nothing) where it is not provided:
// per-point operators and p > 1.
template <typename T>
bool launch_resid_restrict(int p, const DevOp<T>& op, const V2<T>* x, Addr ax, const V2<T>* f,
                           Addr af, int Mc, const T* rw, V2<T>* yc, Addr ac, int nbatch,
                           hipStream_t st);
// The same for per-point operators (op.pn = 1); called by launch_stencil.
template <typename T, typename TX, typename TF, typename TY>
void launch_stencil_pn(int p, int mode, const DevOp<T>& op, const V2<TX>* x, Addr ax,
                       const V2<TF>* f, Addr af, V2<TY>* y, Addr ay, int nbatch, hipStream_t st);
// y = wdinv * f (the first sweep from a zero guess).
template <typename T, typename TF>
void launch_jacobi0(int p, const DevOp<T>& op, const V2<TF>* f, Addr af, V2<T>* y, Addr ay,
                    int nbatch, hipStream_t st);
// yc = P^T r (fine -> coarse), yf (+)= P xc (coarse -> fine).
template <typename T>
void launch_restrict(int p, int Mf, int Mc, const T* rw, const V2<T>* r, V2<T>* yc, int nbatch,
                     Addr af, Addr ac, hipStream_t st);
template <typename T>
void launch_prolong(int p, int Mf, int Mc, const T* rw, const V2<T>* xc, V2<T>* yf, bool add,
                    int nbatch, Addr af, Addr ac, hipStream_t st);
// Per-point operators from per-cell k and shift (heterogeneous k), on a level of order p with
// r x r fine cells per level cell and M lattice points per side; kc [nf*nf] real, sc [nf*nf]
// complex shift multipliers (nullptr: s = 1), nf = r (M - 1) / p fine cells per side.
// Writes A [(2p+1)^2][M*M] and, when wd is given, wd = omega / diag(A).
void launch_assemble_cells(int p, int r, int M, const double* tabK, const double* tabM,
                           const double* tabB, const double* kc, const double2* sc,
                           double omega, double2* A, double2* wd, hipStream_t st);
// Load vector of the point source f = amp exp(-width |x - x_s|^2) (g = 0) on the fine lattice:
// F_i = sum over the triangles T around point i of the quadrature of f phi_i on T.
void launch_gauss_rhs(int p, int n, double sx, double sy, double amp, double width,
                      const double* qxi, const double* qeta, const double* qw,
                      const double* qphi, const int* qloc, int nq, double2* F, hipStream_t st);
// Plane-wave impedance load vector.
void launch_planewave(int p, int n, double k, double theta, const double* gl_t,
                      const double* gl_w, const double* lag, double2* F, hipStream_t st);
// Conversions.
void launch_d2f(const double2* x, float2* y, long n, hipStream_t st);
void launch_d2f_b(const double2* x, Addr ax, float2* y, Addr ay, long n, int nbatch, hipStream_t st);
void launch_f2d(const float2* x, double2* y, long n, hipStream_t st);

// Coarse factorisation: assembles and inverts every block in sequence. Returns HZ_OK or
// HZ_ESINGULAR (pivot check on device, read back at the end).
struct CoarseFactorWork {
  double2* T = nullptr;      // temp blocks, 2 x (max block size)^2 (one per chain)
  double2* W = nullptr;      // pivot row panels, 2 x sweep_panel_elems(max block size)
  double2* R = nullptr;      // pivot block inverses, 2 x sweep_pinv_elems()
  int* flag = nullptr;       // device error flag
};
// Elements of one chain's pivot row panels (two passes' worth) and pivot inverses.
size_t sweep_panel_elems(size_t nmax);
size_t sweep_pinv_elems();
hz_status coarse_factor(const CoarseLayout& L, const DevOp<double>& cop, double2* S,
                        const CoarseFactorWork& w, hipStream_t st);
// Solves A_c y = b with the stored inverses; nrhs right-hand sides with stride cstride.
// Runs as one persistent cooperative launch when possible (workgroups wait for each other's
// block results through sentinel-initialised buffers), else one launch per block row.
struct CoarseSolveWork {
  void* g = nullptr;         // forward-sweep results, 4 right-hand sides x coarse dofs
  int* err = nullptr;        // set to 1 if a wait for another workgroup's data timed out
  bool persistent = true;
};
// One coarse system of a multi-problem solve launch: the problem's factor and coarse stencil
// table, nrhs right-hand sides at b + h cstride, solutions at y + h cstride and a forward-sweep
// buffer at gbuf + h Nc (distinct per job). Up to kMaxJobs jobs of one mesh class share one
// launch, each on its own set of workgroups; jobs are passed by value (kernel arguments).
// ------------------------------------------------------------------------------------------
// Multifrontal coarse factor (nested dissection of the coarse lattice)
// ------------------------------------------------------------------------------------------
//
// The coarse lattice is cut recursively by lattice lines at cell boundaries (points on both
// sides of such a line share no element, so the line separates them) until a region holds at
// most kMfLeaf points. Tree node v owns the points I_v (its separator line, or all points of a
// leaf region) and sees B_v, the points of ancestors' separators on the ring around its
// region. With F_v the frontal matrix on I_v + B_v (the rows of A_c at I_v plus the children's
// update matrices), the factor stores S_v = F_II^{-1}, G_v = S_v F_IB (s x m) and its transpose,
// and passes U_v = F_BB - F_BI G_v to the parent.
constexpr int kMfLeaf = 16;
struct MfNode {
  int s = 0, m = 0;            // |I_v|, |B_v|
  int ch0 = -1, ch1 = -1;      // children
  long Ioff = 0, Boff = 0;     // points of I_v in I[], of B_v in B[]
  long Soff = 0, Goff = 0, GToff = 0;   // S (s x s), G (s x m), G^T (m x s) in the factor
  long uoff = 0;               // update vector (m) in the per-right-hand-side work
  long mapoff = -1;            // front positions in the parent of this node's B points
  long invoff = -1;            // per front position: the child 0 and child 1 entries landing
                               // there (2 ints, -1 for none), for nodes with children
};
// One unit of a solve pass at one tree height: rows [r0, r1) of matrix `kind` of node v
// (kind 0: S, 1: G^T for the forward pass; 2: G for the backward pass; one wave per row), or
// rows [r0, r1) of [S; G^T] of node v, one thread per row (kind 5, forward, s <= 64), or,
// for kinds 3 (forward) and 4 (backward), the whole small nodes hn[r0 .. r1) (one wave each).
struct MfTask {
  int v, kind, r0, r1;
};
// One node of a bottom subtree: factor offsets, |I_v|, |B_v|, the offsets of its points, its
// inverse map (-1 for a leaf) and ring entries within the subtree's, and the LDS offsets of
// its children's and its own update vectors (-1: leaf / the subtree's root).
struct MfSubNode {
  long so, go, gto;
  int s, m, pI, pinv, pB, lu0, lu1, lu;
};
// One bottom subtree: its records sub_node[q0 .. q0 + nrec), points I[i0 .. i0 + np), inverse
// map entries inv[inv0 .. inv0 + ninv), ring entries B[b0 .. b0 + nbm) (the root's, last, are
// mroot at uoff_root in the update vectors) and their local indices sub_bloc[bl0 ..).
struct MfSubHdr {
  long uoff_root = 0, i0 = 0, inv0 = 0, b0 = 0, bl0 = 0;
  int q0 = 0, nrec = 0, np = 0, ninv = 0, nbm = 0, mroot = 0;
};
struct MfSym {
  int p = 1, nc = 0, Mc = 0, H = 0;
  std::vector<MfNode> nodes;              // postorder: children before their parent
  std::vector<int> parent, height;
  std::vector<int> I, B, map, inv;
  long numel = 0, uel = 0;                // factor elements, update elements per right-hand side
  double flop = 0;                        // factorisation: 8 (s^3 + 2 s^2 m + m^2 s) per node
  std::vector<std::vector<int>> at;       // nodes of each height
  std::vector<int> hn;                    // the same, concatenated by height
  std::vector<MfTask> fwd, bwd;           // solve tasks, grouped by height
  std::vector<int> fwd0, bwd0;            // first task of each height (H + 2 entries)
  // Bottom subtrees: the heights 0 .. T (every node small, T <= 3) run as one launch per pass,
  // one workgroup per subtree rooted at a node of height <= T whose parent is higher (its
  // nodes are consecutive in postorder, so are their points, ring lists and inverse maps).
  // sub_node holds each subtree's nodes by ascending height, sub_lev the first of each height
  // 0 .. T + 1 per subtree, sub_bloc per ring entry of a subtree's nodes its index in the
  // subtree's local vector (its points, then the root's ring).
  int T = -1;
  std::vector<MfSubHdr> sub_hdr;
  std::vector<MfSubNode> sub_node;
  std::vector<int> sub_lev;               // nsub * (T + 2)
  std::vector<int> sub_bloc;
  MfSubHdr sub_max;                       // per field, the largest over the subtrees
  int sub_lds = 0;                        // largest update storage of a subtree (elements)
  int maxf = 0;                           // largest s + m
  std::vector<int> fmax, bmax;            // per height: largest s + m, m of a non-small node
  std::vector<char> fbig, bbig;           // per height: prefetch rows (all tasks one wave per
                                          // row, and at most 768 of them)
};
// The (cached) symbolic factor of the coarse lattice of order p with nc cells per side.
const MfSym& mf_symbolic(int p, int nc);
// Device copy of the symbolic data one problem uses.
struct MfView {
  const MfNode* nodes = nullptr;
  const int* I = nullptr;
  const int* B = nullptr;
  const int* map = nullptr;
  const MfTask* fwd = nullptr;
  const MfTask* bwd = nullptr;
  const int* hn = nullptr;
  const int* inv = nullptr;
  const MfSubHdr* sub_hdr = nullptr;
  const MfSubNode* sub_node = nullptr;
  const int* sub_lev = nullptr;
  const int* sub_bloc = nullptr;
};

template <typename T> struct CoarseJob {
  const V2<T>* S = nullptr;
  const V2<T>* coef = nullptr;
  const V2<T>* b = nullptr;
  V2<T>* y = nullptr;
  V2<T>* gbuf = nullptr;
  int nrhs = 1;
  int pn = 0;              // coef holds one stencil per coarse point (as DevOp::pn)
  const MfView* mf = nullptr;   // multifrontal factor: S is its numeric array, gbuf the
                                // update vectors (uel per right-hand side, stride ustride)
  long ustride = 0;
};
constexpr int kMaxJobs = 16;
template <typename T> struct CsJobs {
  CoarseJob<T> j[kMaxJobs];
};
// Largest number of right-hand sides one job may carry for this layout (4, 2 or 1).
template <typename T> int coarse_group(const CoarseLayout& L);
// Solves every job (launches of up to kMaxJobs jobs); returns the number of launches.
template <typename T>
int coarse_solve_jobs(const CoarseLayout& L, const CoarseJob<T>* jobs, int njobs, long cstride,
                      int* err, bool persistent, hipStream_t st);
// Returns the number of solve launches (one reads the factor once for up to 4 right-hand
// sides when their staging fits in LDS).
template <typename T>
int coarse_solve(const CoarseLayout& L, const DevOp<T>& cop, const V2<T>* S, const V2<T>* b,
                 V2<T>* y, int nrhs, long cstride, const CoarseSolveWork& w, hipStream_t st);
void launch_factor_to_f32(const double2* S, float2* Sf, size_t n, hipStream_t st);
// In-place inverse of a complex symmetric n x n row-major block by the symmetric Gauss-Jordan
// sweep (W: 2 sweep_panel_elems(n), R: 2 sweep_pinv_elems() elements of work); sets *flag on a
// zero or non-finite pivot.
void sweep_inverse(double2* X, int n, double2* W, double2* R, int* flag, hipStream_t st);
// The same for nz blocks at once (one launch per pass for all): block z is the n x n matrix at
// base + zs[z].xoff with T = ceil(n / 32) tiles, its panel work at W + zs[z].woff
// (sweep_panel_elems(n) elements) and R + zs[z].roff (sweep_pinv_elems()); maxT the largest T.
struct SweepNode {
  long xoff, woff, roff;
  int n, T;
};
void sweep_inverse_batch(double2* base, const SweepNode* zs, int nz, int maxT, double2* W,
                         double2* R, int* flag, hipStream_t st);
// Device copy of the symbolic data (and of the factorisation's launch tables) of a mesh
// class on the current device, built on first use with stream st and kept until the process
// ends; returns the view on the device and, in host_copy, the same view held on the host.
MfView* mf_device_view(const MfSym& sym, MfView* host_copy, hipStream_t st);
// Multifrontal factorisation of the coarse operator cop into F (sym.numel elements) on the
// device; returns HZ_OK or HZ_ESINGULAR.
hz_status mf_factor(const MfSym& sym, const DevOp<double>& cop, double2* F, int* flag,
                    hipStream_t st);
// Multifrontal solves of njobs jobs (one mesh class; b, y coarse vectors with stride cstride
// per right-hand side, update vectors at gbuf with stride ustride). Returns the launch count.
template <typename T>
int mf_solve_jobs(const MfSym& sym, const CoarseJob<T>* jobs, int njobs, long cstride,
                  hipStream_t st);
// Creates the per-device event that orders persistent coarse-solve launches (otherwise made
// by the first such launch on the device).
void coarse_order_init(int dev);
// Stencil launches of the calling thread pick a variant without timing any (the cached
// choice, else variant 0; every variant gives the same result) while this is off.
void set_stencil_tuning(bool on);

// Krylov kernels. Vectors of length N; a basis V is row-major [nv][ldv].
// Batched forms run nbatch independent instances: instance z uses V + av.at(z), w + aw.at(z),
// its partial sums at partial + z nblk 64 (block b's sums at b 64), its small vectors (h, y)
// at z hs, and its own vector count nvt[z] when the table is given (0 = nothing to do), else
// nv. For launch_maxpy(_b) and launch_maxpy_mdot_b nv bounds the per-instance counts: they
// keep up to nv (<= 64) basis entries per element in registers.
int mdot_blocks(long N);      // blocks (partial sums) of launch_mdot(_b)
int fused_blocks(long N);     // blocks (partial sums) of launch_maxpy(_b), launch_maxpy_mdot_b
// w -= V h, then partial sums of V^H w (the new w) from the same read of V.
void launch_maxpy_mdot_b(const double2* V, Addr av, long ldv, int nv, const int* nvt,
                         const double2* h, long hs, double2* w, Addr aw, long N,
                         double2* partial, int nbatch, hipStream_t st);
void launch_mdot_b(const double2* V, Addr av, long ldv, int nv, const int* nvt, const double2* w,
                   Addr aw, long N, double2* partial, int nblk, int nbatch, hipStream_t st);
// out[z hs + i] = sum over the nblk partial sums of vector i (i < nvt[z], else nv), in a fixed
// order, through work [nbatch][kReduceGroups][64].
constexpr int kReduceGroups = 128;
void launch_reduce_b(const double2* partial, int nblk, int nv, const int* nvt, double2* out,
                     long hs, int nbatch, double2* work, hipStream_t st);
// w -= V h (h on device, nv entries); optionally |w|^2 partials (index 0 of fused_blocks(N)
// blocks).
void launch_maxpy_b(const double2* V, Addr av, long ldv, int nv, const int* nvt, const double2* h,
                    long hs, double2* w, Addr aw, long N, double2* norm_partial, int nbatch,
                    hipStream_t st);
// v = s[z] w (per-instance factor on the device)
void launch_scale_b(const double2* w, Addr aw, const double* s_dev, double2* v, Addr av, long N,
                    int nbatch, hipStream_t st);
// u += Z y (y on the device, nz entries)
template <typename TZ>
void launch_update_b(const V2<TZ>* Z, Addr az, long ldz, int nz, const int* nzt, const double2* y,
                     long ys, double2* u, Addr au, long N, int nbatch, hipStream_t st);
void launch_copy_b(const double2* x, Addr ax, double2* y, Addr ay, long N, int nbatch,
                   hipStream_t st);
void launch_scale_dev(const double2* w, const double* s_dev, double2* v, long N, hipStream_t st);
void launch_scale(const double2* w, double s, double2* v, long N, hipStream_t st);
void launch_fill_zero(double2* y, long N, hipStream_t st);
void launch_fill_zero(float2* y, long N, hipStream_t st);
void launch_fill_zero_b(double2* y, Addr ay, long N, int nbatch, hipStream_t st);
template <typename TZ>
void launch_update(const V2<TZ>* Z, long ldz, int nz, const double2* y, double2* u, long N,
                   hipStream_t st);
void launch_axpby_copy(const double2* x, double2* y, long N, hipStream_t st);

// ------------------------------------------------------------------------------------------
// Errors
// ------------------------------------------------------------------------------------------

void set_error(const std::string& msg);

struct HipError {
  hipError_t e;
  std::string where;
};

#define HZ_HIP(call)                                                           \
  do {                                                                         \
    hipError_t _e = (call);                                                    \
    if (_e != hipSuccess) throw ::hz::HipError{_e, #call};                     \
  } while (0)

}  // namespace hz
