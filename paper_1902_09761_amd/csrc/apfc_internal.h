// Internal declarations of the APFC HIP library: device data descriptors, the nodal bulk
// term table and the kernel launchers.  Not part of the public C ABI (include/apfc.h).
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>
#include <cstddef>
#include <type_traits>

namespace apfc {

constexpr int kTX = 64;          // tile width in x = one wave64
constexpr int kBlock = 256;      // threads per workgroup (4 wave64)
constexpr int kChunk = 2048;     // elements of a full vector per Krylov workgroup (8 per thread)
constexpr int kMaxJ = 8;
constexpr int kMaxTerms = 24;
constexpr int kMaxRestart = 32;
constexpr int kMaxCheb = 64;     // Chebyshev iterations per inner solve
constexpr int kMassRMax = 4;     // taps per side of the separable mass inverse
// bricks of the separable mass inverse and of the 3D Chebyshev L solves: 64 x kMassBY nodes per plane,
// 512 threads; in 3D kBrickZShallow or kBrickZDeep planes (Dev::mbz)
constexpr int kMassBY = 8, kMassThreads = 512;
constexpr int kBrickZShallow = 8, kBrickZDeep = 16;

// Complex value stored as two reals (re, im), 2*sizeof(R)-aligned for vector loads.
template <typename R>
struct alignas(2 * sizeof(R)) cx {
    R x, y;
};
using zd = cx<double>;
using zf = cx<float>;

// One linear system = (instance, amplitude).  Systems are ordered instance-major (s = inst*J + j).
struct Sys {
    int inst, j, dim, nx, ny, nz;
    int tbeg, tend;        // stencil tiles of this system [tbeg, tend)
    int cbeg, cend;        // Krylov chunks of this system [cbeg, cend)
    long long N;           // nodes
    long long off;         // node offset of this system inside a batched half vector
    long long doff;        // node offset of the instance inside per-instance node arrays
    double h, w, kappa, kv[3];
    double a0, a1, a2, a3;
    // time-step dependent scalars (refreshed when dt changes)
    double inv_dt, isq_dt, sq_kap, isq_kap;
    double diagM, diagK, diagL;
    // Chebyshev parameters (centre theta, half width delta) of the Jacobi-scaled spectra of M and
    // L = M/sqrt(dt) + sqrt(kappa) K on the periodic uniform mesh
    double thM, deM, thL, deL;
    // Chebyshev scalars of the two inner operators (0: M, 1: L), folded with the Jacobi diagonal D:
    // cb[op][0][0] = 1/(theta D) (d_0 = cb r_0), and for j >= 1 cb[op][j] = {rho_j rho_{j-1}, 2 rho_j/(delta D)}
    // with rho_0 = delta/theta, rho_j = 1/(2 theta/delta - rho_{j-1}).  Indexed dynamically, so kernels
    // read it through the Sys pointer, not from a local copy.
    double cb[2][kMaxCheb][2];
    // 1D taps of the separable mass inverse, wsep[k] = (sqrt(3)/h) rho^k, rho = sqrt(3) - 2 (k <= kMassRMax)
    double wsep[kMassRMax + 1];
};

struct Tile { int sys, x0, y0, z; };
// Interior tile of the fused Chebyshev preconditioner kernels (region = interior + halo).
struct CTile { int sys, x0, y0, z; };
// LDS region shapes (width, height, threads) of the fused preconditioner kernels; every thread owns
// height * width / threads consecutive rows of one column.
constexpr int kChebShapes = 6;
constexpr int kChebShape[kChebShapes][3] = {{128, 32, 512}, {64, 32, 256}, {64, 64, 512},
                                            {128, 36, 512}, {128, 64, 1024}, {256, 32, 1024}};

struct Chunk { int sys; int e0; };     // element offset inside the system's 2N-element full vector

// Resonant products of the bulk energy with distinct amplitude indices: term value
// c (T + T^*), T = prod_q u_q, u_q = eta_{idx[q]} or its conjugate (cj[q] = 1); c = -2 a3/a0
// for cubic terms (order 3) and 8 a2/a0 for quartic ones (order 4).
struct Terms {
    int J;
    int n;
    int order[kMaxTerms];
    int idx[kMaxTerms][4];
    int cj[kMaxTerms][4];
};

// Reduction slots in the per-tile partial array (stride kSlots).
enum Slot { kRho0 = 0, kRho1 = 1, kPQ = 2, kRR = 3, kBB = 4, kE0 = 5, kE1 = 6, kSlots = 8 };

// Kernel identifiers for the timing probe.
enum KernelId {
    KID_ALL = -2, KID_NONE = -1, KID_PCG_SPMV = 0, KID_PCG_UPDATE, KID_PCG_INIT, KID_PC_FINAL, KID_APPLY,
    KID_RESIDUAL, KID_GS, KID_PROJ_FINAL, KID_XUPDATE, KID_REDUCE, KID_SMALL, KID_OTHER, KID_CHEB, KID_EXTRAP,
    KID_RHS, KID_MG, KID_MASS, KID_COUNT
};
const char* kernel_name(int kid);
int kernel_id(const char* name);

struct Probe {
    int target = KID_NONE;    // one kernel family, or KID_ALL: every family, each sampled on its own
    int n = 0;
    int every = 1;            // record every `every`-th launch of the target (of each family with KID_ALL)
    long long seen[KID_COUNT] = {};   // launches per family since the probe was enabled
    static constexpr int kMax = 8192;
    hipEvent_t ev[2 * kMax];
    int kid[kMax];              // family of recorded launch i
    double bytes[kMax];         // algorithmic HBM bytes of recorded launch i with every system active
    double* d_frac = nullptr;   // device [kMax]: share of the nodes whose systems launch i worked on
    bool created = false;
};

// Everything a launcher needs about the batch (device pointers + host copies of sizes).
struct Dev {
    const Sys* sys = nullptr;        // device [S]
    const Tile* tiles = nullptr;     // device [ntiles]
    const Chunk* chunks = nullptr;   // device [nchunks]
    const Tile* mtiles = nullptr;    // device [nmtiles]: bricks of the separable mass inverse
    int nmtiles = 0, mbz = kBrickZShallow;   // brick depth in planes (3D)
    int ntiles = 0, nchunks = 0, S = 0, TY = 16, J = 0, count = 0, dim = 2;
    long long NT = 0;                // half-vector length (complex values)
    Terms terms{};
    Probe* probe = nullptr;
};

// Calls f(std::integral_constant<int, depth>{}) with the brick depth of d.
template <typename F>
void brick_depth(const Dev& d, const F& f) {
    if (d.mbz == kBrickZDeep)
        f(std::integral_constant<int, kBrickZDeep>{});
    else
        f(std::integral_constant<int, kBrickZShallow>{});
}

// Levels of the multigrid inner solve below the fine one (APFC_INNER_MG): level l + 1 of the V-cycle is
// lev[l] (its own Sys and tile tables, 16-row tiles) with its buffers in the storage precision.
constexpr int kMgMaxLevels = 16;
constexpr int kMgCoarseMax = 8192;   // nodes of a system on the coarsest level (solved in LDS)
struct MgLevels {
    int n = 0;
    Dev lev[kMgMaxLevels];
    void *x[kMgMaxLevels] = {}, *b[kMgMaxLevels] = {}, *r[kMgMaxLevels] = {}, *d0[kMgMaxLevels] = {},
         *d1[kMgMaxLevels] = {};
    int nu = 2;             // Chebyshev smoothing iterations before and after the coarse correction
    int coarse_its = 24;    // Chebyshev iterations on the coarsest level
};

// Krylov bookkeeping on the device (all [S]-indexed, see api.hip).
struct Krylov {
    double* H;          // [S][m][m+1] complex, column k holds rows 0..k after the rotations
    double* cs;         // [S][m]
    double* sn;         // [S][m] complex
    double* g;          // [S][m+1] complex
    double* y;          // [S][m] complex
    double* hsum;       // [S][m+1] complex, h1 + h2 of the current column
    double* hinv;       // [S] 1/||w''||
    double* red1;       // [S][nv1+1] reduction scratch (autotuner)
    double* redr;       // [S][2] reduced |r|^2, |b|^2
    double* bnorm;      // [S]
    double* target;     // [S]
    double* inv_beta;   // [S]
    double* relres;     // [S]
    int* solve_active;  // [S]
    int* iter_active;   // [S]
    int* reorth;        // [S] second Gram-Schmidt pass needed in this iteration
    int always_reorth;  // 1: classical Gram-Schmidt twice on every iteration
    double reorth_theta;  // second pass when |w'|^2 < reorth_theta |w|^2
    int* kcount;        // [S]
    int* iters;         // [S]
    int* cycles;        // [S]
    int* err;           // [1]
    int* tick_c;        // [S] chunks of the system done in the current second-pass launch
    int* tick_p;        // [1] workgroups done in the current cycle-start launch
    int m;
    int nv1;            // 2*(m+1)
    double rtol;
};

// ------------------------------------------------------------------------------------------
// Launchers (kernels.hip).  `mask` points to per-system int flags (nullptr = all systems).
// ------------------------------------------------------------------------------------------
void launch_state_in(const Dev& d, double* const* eta_tab, double* const* zeta_tab, zd* X, hipStream_t st);
void launch_state_out(const Dev& d, const zd* X, double* const* eta_tab, double* const* zeta_tab, hipStream_t st);
void launch_planar_in(const Dev& d, double* const* tab, zd* half, hipStream_t st);
void launch_planar_out(const Dev& d, const zd* half, double* const* tab, hipStream_t st);
void launch_fill_zero(zd* p, long long n, hipStream_t st);
// k_rhs_base + k_nonlinear in one pass (K = 1)
void launch_rhs_nonlinear(const Dev& d, const zd* eta_half, double* const* src_tab, double* dnode, zd* B,
                          hipStream_t st);
void launch_extrapolate(const Dev& d, const zd* X, const zd* const* h, zd* X0, zd* keep, int order,
                        hipStream_t st);
void launch_widen(const zf* in, zd* out, long long n, hipStream_t st);
void launch_narrow(const zd* in, zf* out, long long n, hipStream_t st);

void launch_rhs_base(const Dev& d, const zd* Xeta, double* const* src_tab, zd* BB, hipStream_t st);
void launch_nonlinear(const Dev& d, const zd* eta_half, const zd* BB, double* dnode, zd* B, hipStream_t st);

template <typename RT>
void launch_residual(const Dev& d, const zd* X, const zd* B, const double* dnode, RT* R, double* part,
                     const int* mask, hipStream_t st);
template <typename T>
void launch_apply(const Dev& d, const cx<T>* Z, const double* dnode, zd* W, const int* mask, hipStream_t st);

template <typename T>
void launch_precond(const Dev& d, const cx<T>* v, cx<T>* z, cx<T>* x1, cx<T>* x2, cx<T>* r, cx<T>* p0, cx<T>* p1,
                    cx<T>* q, double* part, int mass_iters, int diff_iters, int mass_sep, const int* mask,
                    hipStream_t st);

// mass_sep > 0 (every preconditioner launcher): step 1 by the separable mass inverse with mass_sep taps per
// side (launch_mass_sep) instead of mass_iters inner iterations.
// vscale (may be null): the input is vscale[sys] * rv instead of v, and that scaled vector is also
// stored to vout
// Input of the fused 2D preconditioner formed as it is loaded (a basis vector of FGMRES) instead of read:
// v = (src - sum_{l < nv} c_l V_l) * scale[sys] with c_l = hcoef[sys * hld + 2l] + i hcoef[sys * hld + 2l + 1],
// in FP64 from the stored values, and stored to vout at the nodes each region owns.  src = null: v is read.
template <typename T>
struct VIn {
    const cx<T>* src = nullptr;
    const cx<T>* V = nullptr;   // V_l at V + l * vs
    long long vs = 0;
    int nv = 0;
    const double* hcoef = nullptr;
    int hld = 0;
    const double* scale = nullptr;
    cx<T>* vout = nullptr;
};

template <typename T>
void launch_precond_cheb(const Dev& d, int shape, const CTile* ctiles, int nctiles, int halo, const cx<T>* v,
                         cx<T>* z, cx<T>* x1, cx<T>* x2, int mass_iters, int diff_iters, int mass_sep,
                         const VIn<T>& vin, const int* mask, hipStream_t st);

template <typename T>
void launch_precond_cheb_unfused(const Dev& d, const cx<T>* v, cx<T>* z, cx<T>* x1, cx<T>* x2, cx<T>* r, cx<T>* d0,
                                 cx<T>* d1, int mass_iters, int diff_iters, int mass_sep, const int* mask,
                                 hipStream_t st);
// Workgroups of the 3D brick Chebyshev iteration (bricks of bz planes, FP32 when single) that one compute
// unit holds at once; 0 if the runtime cannot tell.
int brick_occupancy(int bz, bool single);
// x1 = W beta1 (beta1 = the zeta part of v): the separable approximate inverse of the mass matrix, taps
// Sys::wsep[0..R] in every direction, on the bricks d.mtiles (kernels_mass.hip).
template <typename T>
void launch_mass_sep(const Dev& d, int R, const cx<T>* v, cx<T>* x1, const int* mask, hipStream_t st);

void launch_reduce(const Dev& d, const double* part, int slot0, int nvals, bool chunk_ranges, double* out, int ld,
                   const int* mask, hipStream_t st);
// Both Gram-Schmidt passes of Arnoldi step k: the first from the operator apply's per-tile partials
// part1, the second (only for the systems that need it) into part2; then the Hessenberg column.
template <typename VT>
void launch_gs(const Dev& d, const Krylov& kr, int k, const double* part1, const VT* V, long long vstride,
               const VT* w, double* part2, hipStream_t st);
template <typename T>
void launch_apply_dot(const Dev& d, const cx<T>* Z, const double* dnode, cx<T>* W, const cx<T>* V, long long vstride, int nv,
                      double* part, const int* mask, hipStream_t st);
template <typename VT>
void launch_proj_final(const Dev& d, const VT* V, long long vstride, int nv, const VT* w, const double* hcoef,
                       const double* hinv, int hstride, VT* out, const int* mask, hipStream_t st);
template <typename VT>
void launch_scale(const Dev& d, const VT* r, const double* inv_beta, VT* v0, const int* mask, hipStream_t st);
template <typename T>
void launch_xupdate(const Dev& d, const cx<T>* Z, long long zstride, const int* kcount, const double* y, int ldy,
                    zd* X, const int* mask, hipStream_t st);

// Start of a restart cycle from the residual partials of launch_residual: per-system reduction of
// |r|^2 and |b|^2, beta, target and the cycle's state (first: the solve's start); with pub set, the
// last workgroup also writes the host summary (any system still solving, non-finite flag, largest
// iteration count) to pub.
void launch_cycle_start(const Dev& d, const Krylov& kr, const double* part, bool first, int* pub, hipStream_t st);
void launch_solve_y(const Dev& d, const Krylov& kr, hipStream_t st);

void launch_mass_solve(const Dev& d, const zd* eta, zd* zeta, zd* r, zd* p0, zd* p1, zd* q, double* part,
                       int iters, hipStream_t st);
// One multigrid V-cycle x = V(b) for L on every system (kernels_mg.hip); fine-level work buffers r, d0, d1.
template <typename T>
void launch_mg_vcycle(const Dev& fine, const MgLevels& mg, const cx<T>* b, cx<T>* x, cx<T>* r, cx<T>* d0, cx<T>* d1,
                      const int* mask, hipStream_t st);
// The block preconditioner with the multigrid L solves: step 1 by mass_iters Chebyshev iterations (or the
// separable mass inverse), steps 2 and 3 by one V-cycle each, step 4.
template <typename T>
void launch_precond_mg(const Dev& d, const MgLevels& mg, const cx<T>* v, cx<T>* z, cx<T>* x1, cx<T>* x2, cx<T>* r,
                       cx<T>* d0, cx<T>* d1, cx<T>* b, int mass_iters, int mass_sep, const int* mask,
                       hipStream_t st);
void launch_energy_parts(const Dev& d, const zd* eta, const zd* zeta, double* part, hipStream_t st);
void launch_energy_grad(const Dev& d, const zd* eta, const zd* zeta, double* const* grad_tab, double* part,
                        hipStream_t st);
struct RefineArgs {
    double inv_KtK[3][3];      // (sum_j k_j k_j^T)^{-1} is formed per node; kmax = max_j |k_j|
    double kmax, nwl, eps, Amin, hint, hmax, tiny;
};
void launch_rotation(const Dev& d, const zd* eta, double* const* omega_tab, double* const* h_tab, const RefineArgs& ra,
                     hipStream_t st);
void launch_adjoint_rhs(const Dev& d, double* const* lam_tab, zd* B, hipStream_t st);
void launch_adjoint_out(const Dev& d, const zd* Y, const zd* eta_prev, double* const* eta_new_tab,
                        double* const* lam_out_tab, double* part, hipStream_t st);

}  // namespace apfc
