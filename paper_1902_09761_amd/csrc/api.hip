// Host side of the APFC library: argument checking, batch tables, workspace carving, the
// restarted FGMRES driver of the per-amplitude block systems (Algorithm 1, Eq. (10)-(12)),
// energy, gradient and adjoint entry points, the timing probe, the tile autotuner and hipGraph
// capture of FGMRES iterations.  Every device buffer belongs to the caller.
#include "apfc.h"
#include "apfc_internal.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdint>
#include <cstring>
#include <string>
#include <vector>

using namespace apfc;

namespace {

thread_local std::string g_err;

int fail(int code, const std::string& msg) {
    g_err = msg;
    return code;
}

#define HIPCHK(expr)                                                                                 \
    do {                                                                                             \
        hipError_t e_ = (expr);                                                                      \
        if (e_ != hipSuccess) return fail(APFC_ERR_HIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
    } while (0)

// ----------------------------------------------------------------------------------------------
// Resonant products of the bulk energy (Eq. (1), (5)): the part of <n^p> (p = 3, 4) that survives
// the average over the lattice scale.  With distinct amplitude indices the ordered products of a
// set occur p! times; pair terms |eta_i|^2 |eta_l|^2 give A^2 - 2 sum |eta|^4 of Eq. (5).
// ----------------------------------------------------------------------------------------------
bool zero_vec(const double* v) { return std::fabs(v[0]) < 1e-9 && std::fabs(v[1]) < 1e-9 && std::fabs(v[2]) < 1e-9; }

int build_terms(const apfc_lattice& L, Terms& T) {
    std::memset(&T, 0, sizeof(T));
    T.J = L.J;
    const int J = L.J;
    // distinct-index resonances, first factor unconjugated (its conjugate is the "+ c.c." part)
    for (int order = 3; order <= 4; ++order) {
        int idx[4];
        for (idx[0] = 0; idx[0] < J; ++idx[0])
            for (idx[1] = idx[0] + 1; idx[1] < J; ++idx[1])
                for (idx[2] = idx[1] + 1; idx[2] < J; ++idx[2])
                    for (int i3 = (order == 4 ? idx[2] + 1 : 0); i3 < (order == 4 ? J : 1); ++i3) {
                        idx[3] = i3;
                        for (int signs = 0; signs < (1 << (order - 1)); ++signs) {
                            double v[3] = {0, 0, 0};
                            int cj[4] = {0, 0, 0, 0};
                            for (int q = 0; q < order; ++q) {
                                cj[q] = q == 0 ? 0 : (signs >> (q - 1)) & 1;
                                for (int c = 0; c < 3; ++c) v[c] += (cj[q] ? -1.0 : 1.0) * L.k[idx[q]][c];
                            }
                            if (!zero_vec(v)) continue;
                            if (T.n >= kMaxTerms) return fail(APFC_ERR_INVALID, "lattice: too many resonant terms");
                            T.order[T.n] = order;
                            for (int q = 0; q < order; ++q) {
                                T.idx[T.n][q] = idx[q];
                                T.cj[T.n][q] = cj[q];
                            }
                            T.n++;
                        }
                    }
    }
    // every other zero-sum product must be a pair term (k_i - k_i + k_l - k_l)
    for (int i = 0; i < J; ++i)
        for (int l = i + 1; l < J; ++l)
            for (int si = -1; si <= 1; si += 2) {
                double v[3];
                for (int c = 0; c < 3; ++c) v[c] = L.k[i][c] + si * L.k[l][c];
                if (zero_vec(v)) return fail(APFC_ERR_INVALID, "lattice: k_l = +-k_i for l != i");
            }
    for (int i = 0; i < J; ++i)
        for (int l = 0; l < J; ++l)
            for (int si = -1; si <= 1; si += 2) {
                // 2 k_i +- k_l = 0 (cubic with a repeated index)
                double v[3];
                for (int c = 0; c < 3; ++c) v[c] = 2.0 * L.k[i][c] + si * L.k[l][c];
                if (zero_vec(v)) return fail(APFC_ERR_INVALID, "lattice: resonance 2 k_i = -+ k_l not supported");
                for (int m = 0; m < J; ++m)
                    for (int sm = -1; sm <= 1; sm += 2) {
                        // 2 k_i + si k_l + sm k_m = 0 (quartic with a repeated index, not a pair term);
                        // l = i or m = i with a minus sign leaves k_i -+ k_other, zero only for |eta_i|^4
                        if ((l == i && si == -1) || (m == i && sm == -1)) continue;
                        for (int c = 0; c < 3; ++c) v[c] = 2.0 * L.k[i][c] + si * L.k[l][c] + sm * L.k[m][c];
                        if (zero_vec(v)) return fail(APFC_ERR_INVALID, "lattice: resonance 2 k_i + k_l + k_m = 0 not supported");
                    }
            }
    return APFC_OK;
}

// f^s(phi) = c2 phi^2 + c3 phi^3 + c4 phi^4 for the uniform crystal eta_j = phi.
void uniform_poly(const Terms& T, const apfc_params& p, double& c2, double& c3, double& c4) {
    const int J = T.J;
    c2 = 2.0 * J * p.a1 / p.a0;                                  // (a1/a0) A, A = 2 J phi^2
    c4 = p.a2 / p.a0 * (4.0 * J * J - 2.0 * J);                  // (a2/a0)(A^2 - 2 sum |eta|^4)
    c3 = 0.0;
    for (int t = 0; t < T.n; ++t) {
        if (T.order[t] == 3) c3 += 2.0 * (-2.0 * p.a3 / p.a0);
        else c4 += 2.0 * (8.0 * p.a2 / p.a0);
    }
}

}  // namespace

// ----------------------------------------------------------------------------------------------
// context
// ----------------------------------------------------------------------------------------------
struct apfc_ctx {
    int count = 0, J = 0, dim = 2, S = 0;
    apfc_lattice lattice{};
    std::vector<apfc_mesh> meshes;
    std::vector<apfc_params> params;
    apfc_params solver{};
    Terms terms{};
    std::vector<Sys> sys;
    std::vector<Tile> tiles;
    std::vector<Chunk> chunks;
    std::vector<CTile> ctiles;
    CTile* d_ctiles = nullptr;
    std::vector<Tile> mtiles;          // bricks of the separable mass inverse and the 3D Chebyshev L solves
    int mbz = kBrickZShallow;          // their depth in planes (3D)
    Tile* d_mtiles = nullptr;
    int cheb_shape = 0;
    size_t max_ctiles = 0;
    long long NT = 0, NI = 0;
    int TY = 16;
    int max_tiles = 0;
    double dt = -1.0;
    bool mixed = false;
    // multigrid inner solve (APFC_INNER_MG): the levels below the fine one, each with its own system and
    // tile tables and five work vectors (x, b, r, d0, d1) in the preconditioner precision
    int mg_n = 0;
    std::vector<Sys> mg_sys[kMgMaxLevels];
    std::vector<Tile> mg_tiles[kMgMaxLevels];
    long long mg_NT[kMgMaxLevels] = {};
    Sys* d_mg_sys[kMgMaxLevels] = {};
    Tile* d_mg_tiles[kMgMaxLevels] = {};
    void* mg_buf[kMgMaxLevels][5] = {};

    // workspace: ws is the memory the buffers below are carved from, either the caller's workspace
    // (ws_user, apfc_set_workspace) or, during and after apfc_step_noalloc, the static scratch
    char* ws = nullptr;
    size_t ws_bytes = 0;
    char* ws_user = nullptr;
    size_t ws_user_bytes = 0;
    size_t ws_need = 0;                // bytes carve() needs (fixed at create)
    Sys* d_sys = nullptr;
    Tile* d_tiles = nullptr;
    Chunk* d_chunks = nullptr;
    double** d_tab = nullptr;          // 4 tables of [count] pointers
    zd *X = nullptr, *B = nullptr, *R = nullptr, *W = nullptr, *BB = nullptr;
    zd* V = nullptr;
    void* Z = nullptr;
    void* pc[6] = {};
    double* dnode = nullptr;
    double* tpart = nullptr;
    double* cpart = nullptr;
    double* apart = nullptr;
    Krylov kr{};
    int m = 30;
    int cycle_hint = 0;   // restart cycles of the slowest system in the last solve
    // apfc_run statistics (device, [S])
    long long* run_it_sum = nullptr;
    int *run_it_max = nullptr, *run_cyc_max = nullptr;
    double* run_res_max = nullptr;
    // states passed to the last x0_order steps, for the extrapolated initial guess: a ring of
    // K = x0_order buffers, hist[newest] = x^{m-1}, hist[newest - 1] = x^{m-2}, ...; hist_n valid
    zd* hist[3] = {nullptr, nullptr, nullptr};
    int hist_newest = 0, hist_n = 0;
    double hist_dt = 0.0;

    // host staging (pinned)
    double** h_tab = nullptr;
    std::vector<const void*> tab_shadow;   // pointer tables currently in d_tab
    int* h_flags = nullptr;
    int* h_pub = nullptr;                  // mapped host flags written by k_cycle_start
    int* d_pub = nullptr;
    double* h_dbl = nullptr;
    // apfc_step_noalloc: pageable host staging sized at create (the call allocates nothing) and the
    // device copy of the host summary of k_cycle_start (in the carved memory)
    bool noalloc = false;
    int* pub_dev = nullptr;
    std::vector<const void*> na_ptrs;
    std::vector<double*> na_tab;
    std::vector<int> na_flags;
    std::vector<double> na_dbl;
    int na_pub[8] = {};

    Probe probe;
    bool use_graphs = false;
    hipStream_t cap_stream = nullptr;
    std::vector<hipGraphExec_t> graphs;
    bool graphs_valid = false;

    Dev dev() {
        Dev d;
        d.sys = d_sys;
        d.tiles = d_tiles;
        d.chunks = d_chunks;
        d.mtiles = d_mtiles;
        d.nmtiles = (int)mtiles.size();
        d.mbz = mbz;
        d.ntiles = (int)tiles.size();
        d.nchunks = (int)chunks.size();
        d.S = S;
        d.TY = TY;
        d.J = J;
        d.count = count;
        d.dim = dim;
        d.NT = NT;
        d.terms = terms;
        d.probe = probe.target != KID_NONE ? &probe : nullptr;
        return d;
    }
    size_t zsize() const { return mixed ? sizeof(zf) : sizeof(zd); }
    long long vstride() const { return 2 * NT; }   // complex values per full vector
};

// Drops the context from the owners of the static scratch of apfc_step_noalloc (apfc_destroy).
void noalloc_forget(const apfc_ctx* c);

namespace {

// Workgroups go to the 8 XCDs of the chip in turn (workgroup b to XCD b mod 8), each XCD with its own L2.
constexpr int kXcds = 8;

// Appends tiles in XCD-contiguous order: the workgroups of one XCD take consecutive tiles of the natural
// order, so a tile's neighbours (whose nodes its halo re-reads) sit in the same L2.
template <typename TL>
void append_xcd_order(const std::vector<TL>& nat, std::vector<TL>& out) {
    const int T = (int)nat.size(), per = T / kXcds, rem = T % kXcds;
    for (int l = 0; l < T; ++l) {
        const int x = l % kXcds, q = l / kXcds;
        out.push_back(nat[x * per + std::min(x, rem) + q]);
    }
}

void build_tiles(apfc_ctx& c, int TY, std::vector<Tile>& tiles) {
    tiles.clear();
    for (int s = 0; s < c.S; ++s) {
        Sys& y = c.sys[s];
        y.tbeg = (int)tiles.size();
        if (y.dim == 3) {   // 64 x 4 x TY/4 bricks
            std::vector<Tile> nat;
            for (int z0 = 0; z0 < y.nz; z0 += TY / 4)
                for (int y0 = 0; y0 < y.ny; y0 += 4)
                    for (int x0 = 0; x0 < y.nx; x0 += kTX) nat.push_back(Tile{s, x0, y0, z0});
            append_xcd_order(nat, tiles);
        } else {
            std::vector<Tile> nat;
            for (int y0 = 0; y0 < y.ny; y0 += TY)
                for (int x0 = 0; x0 < y.nx; x0 += kTX) nat.push_back(Tile{s, x0, y0, 0});
            append_xcd_order(nat, tiles);
        }
        y.tend = (int)tiles.size();
    }
}

// Extremes of the Jacobi-scaled symbols of M and L = M/sqrt(dt) + sqrt(kappa) K on the periodic
// uniform mesh.  With c_d = cos(theta_d): M^ = h^dim prod_d (2 + c_d)/3 and
// K^ = h^(dim-2) sum_d (2 - 2 c_d) prod_{e != d} (2 + c_e)/3 are multilinear in (c_1..c_dim), so the
// extremes over [-1, 1]^dim sit at the corners.
void cheb_bounds(const Sys& y, double& thM, double& deM, double& thL, double& deL) {
    double mnM = 1e300, mxM = -1e300, mnL = 1e300, mxL = -1e300;
    for (int corner = 0; corner < (1 << y.dim); ++corner) {
        double cc[3];
        for (int d = 0; d < y.dim; ++d) cc[d] = (corner >> d) & 1 ? -1.0 : 1.0;
        double Mh = std::pow(y.h, y.dim), Kh = 0.0;
        for (int d = 0; d < y.dim; ++d) Mh *= (2.0 + cc[d]) / 3.0;
        for (int d = 0; d < y.dim; ++d) {
            double t = (2.0 - 2.0 * cc[d]) * std::pow(y.h, y.dim - 2);
            for (int e = 0; e < y.dim; ++e)
                if (e != d) t *= (2.0 + cc[e]) / 3.0;
            Kh += t;
        }
        const double lm = Mh / y.diagM, ll = (Mh * y.isq_dt + y.sq_kap * Kh) / y.diagL;
        mnM = std::min(mnM, lm);
        mxM = std::max(mxM, lm);
        mnL = std::min(mnL, ll);
        mxL = std::max(mxL, ll);
    }
    thM = 0.5 * (mxM + mnM);
    deM = 0.5 * (mxM - mnM);
    thL = 0.5 * (mxL + mnL);
    deL = 0.5 * (mxL - mnL);
}

void cheb_table(Sys& y) {
    const double th[2] = {y.thM, y.thL}, de[2] = {y.deM, y.deL}, dg[2] = {y.diagM, y.diagL};
    for (int op = 0; op < 2; ++op) {
        const double sig = th[op] / de[op];
        double rho = 1.0 / sig;
        y.cb[op][0][0] = 1.0 / (th[op] * dg[op]);
        y.cb[op][0][1] = 0.0;
        for (int j = 1; j < kMaxCheb; ++j) {
            const double rn = 1.0 / (2.0 * sig - rho);
            y.cb[op][j][0] = rn * rho;
            y.cb[op][j][1] = 2.0 * rn / (de[op] * dg[op]);
            rho = rn;
        }
    }
}

void sys_dt(Sys& y, double dt) {
    y.inv_dt = 1.0 / dt;
    y.isq_dt = 1.0 / std::sqrt(dt);
    y.sq_kap = std::sqrt(y.kappa);
    y.isq_kap = 1.0 / std::sqrt(y.kappa);
    y.diagL = y.diagM * y.isq_dt + y.sq_kap * y.diagK;
    cheb_bounds(y, y.thM, y.deM, y.thL, y.deL);
    cheb_table(y);
}

// Multigrid smoother: Chebyshev-Jacobi iterations for the upper part [lam_max/alpha, lam_max] of the
// spectrum of D^{-1} L (lam_max = thL + deL), in the L table (cb[1]) of a level that is not the
// coarsest; the coarsest level keeps the whole-spectrum table of cheb_table.
constexpr double kMgAlpha = 4.0;
void mg_smoother_table(Sys& y) {
    const double hi = y.thL + y.deL, lo = hi / kMgAlpha;
    const double th = 0.5 * (hi + lo), de = 0.5 * (hi - lo), sig = th / de;
    double rho = 1.0 / sig;
    y.cb[1][0][0] = 1.0 / (th * y.diagL);
    y.cb[1][0][1] = 0.0;
    for (int j = 1; j < kMaxCheb; ++j) {
        const double rn = 1.0 / (2.0 * sig - rho);
        y.cb[1][j][0] = rn * rho;
        y.cb[1][j][1] = 2.0 * rn / (de * y.diagL);
        rho = rn;
    }
}

void set_dt_scalars(apfc_ctx& c, double dt) {
    for (auto& y : c.sys) {
        sys_dt(y, dt);
        if (c.mg_n > 0) mg_smoother_table(y);
    }
    for (int l = 0; l < c.mg_n; ++l)
        for (auto& y : c.mg_sys[l]) {
            sys_dt(y, dt);
            if (l + 1 < c.mg_n) mg_smoother_table(y);
        }
    c.dt = dt;
}

// 1D taps of the separable mass inverse: the inverse of (h/6) tridiag(1, 4, 1) on an unbounded uniform
// mesh has the entries (sqrt(3)/h) rho^|k| with rho = sqrt(3) - 2 (the root of modulus below one of
// rho^2 + 4 rho + 1 = 0).
void set_wsep(Sys& y) {
    const double rho = std::sqrt(3.0) - 2.0;
    double t = std::sqrt(3.0) / y.h;
    for (int k = 0; k <= kMassRMax; ++k, t *= rho) y.wsep[k] = t;
}

// The multigrid levels (APFC_INNER_MG): coarsen all systems together while every direction of every
// system is even and its half at least kMgCoarseMin nodes (16 in 2D, 8 in 3D); a coarse level is the
// same periodic domain with twice the mesh size.  The coarsest level of each system must hold at most
// kMgCoarseMax nodes (it is solved in LDS).
int build_mg_levels(apfc_ctx& c) {
    const int cmin = c.dim == 3 ? 8 : 16;
    std::vector<Sys> prev = c.sys;
    c.mg_n = 0;
    for (;;) {
        bool ok = c.mg_n + 1 < kMgMaxLevels;
        for (const Sys& y : prev) {
            const int n[3] = {y.nx, y.ny, y.nz};
            for (int d = 0; d < y.dim; ++d) ok = ok && n[d] % 2 == 0 && n[d] / 2 >= cmin;
        }
        if (!ok) break;
        const int l = c.mg_n;
        c.mg_sys[l].clear();
        c.mg_tiles[l].clear();
        long long off = 0;
        for (int si = 0; si < (int)prev.size(); ++si) {
            Sys y = prev[si];
            y.nx /= 2;
            y.ny /= 2;
            if (y.dim == 3) y.nz /= 2;
            y.N = (long long)y.nx * y.ny * y.nz;
            y.off = off;
            off += y.N;
            y.h *= 2.0;
            y.w = std::pow(y.h, y.dim);
            set_wsep(y);
            y.diagM = std::pow(2.0 * y.h / 3.0, y.dim);
            y.diagK = y.dim * (2.0 / y.h) * std::pow(2.0 * y.h / 3.0, y.dim - 1);
            y.tbeg = (int)c.mg_tiles[l].size();
            if (y.dim == 3) {
                for (int z0 = 0; z0 < y.nz; z0 += 4)
                    for (int y0 = 0; y0 < y.ny; y0 += 4)
                        for (int x0 = 0; x0 < y.nx; x0 += kTX) c.mg_tiles[l].push_back(Tile{si, x0, y0, z0});
            } else {
                for (int y0 = 0; y0 < y.ny; y0 += 16)
                    for (int x0 = 0; x0 < y.nx; x0 += kTX) c.mg_tiles[l].push_back(Tile{si, x0, y0, 0});
            }
            y.tend = (int)c.mg_tiles[l].size();
            c.mg_sys[l].push_back(y);
        }
        c.mg_NT[l] = off;
        prev = c.mg_sys[l];
        c.mg_n += 1;
    }
    for (const Sys& y : prev)
        if (y.N > kMgCoarseMax)
            return fail(APFC_ERR_INVALID, "APFC_INNER_MG: a system's coarsest multigrid level has " + std::to_string(y.N) +
                                              " nodes, more than " + std::to_string(kMgCoarseMax) +
                                              " (use mesh sizes that halve further)");
    return APFC_OK;
}

// Halo of the fused 2D Chebyshev regions: stage 0 needs mass_iters - 1 stencil layers (or mass_iters taps of
// the separable mass inverse), stages 1 and 2 one layer for G x1 or M x2 plus diff_iters - 1.
int cheb_halo(const apfc_params& p) {
    return std::max(p.mass_kind == APFC_MASS_SEPARABLE ? p.mass_iters : p.mass_iters - 1, p.diff_iters);
}

// Bricks of the separable mass inverse and of the 3D Chebyshev L solves: 64 x kMassBY nodes per plane;
// in 3D, bz = kBrickZShallow or kBrickZDeep planes, whichever gives the smaller (workgroup rounds) x (bz + 2
// planes marched per brick), a round being as many bricks as the chip holds at once: deeper bricks re-read
// fewer halo planes, but a partly filled last round costs as much as a full one.
void build_mtiles(apfc_ctx& c) {
    c.mtiles.clear();
    if (c.solver.mass_kind != APFC_MASS_SEPARABLE && c.dim != 3) return;
    auto count = [&](int bz) {
        long long n = 0;
        for (int s = 0; s < c.S; ++s) {
            const Sys& y = c.sys[s];
            n += (long long)((y.nx + kTX - 1) / kTX) * ((y.ny + kMassBY - 1) / kMassBY) * ((y.nz + bz - 1) / bz);
        }
        return n;
    };
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        cus = 256;
    auto cost = [&](int bz) {
        const long long slots = (long long)std::max(1, cus) * std::max(1, brick_occupancy(bz, c.mixed));
        return (count(bz) + slots - 1) / slots * (bz + 2);
    };
    c.mbz = c.dim == 3 && cost(kBrickZDeep) < cost(kBrickZShallow) ? kBrickZDeep : kBrickZShallow;
    for (int s = 0; s < c.S; ++s) {
        const Sys& y = c.sys[s];
        std::vector<Tile> nat;
        for (int z0 = 0; z0 < y.nz; z0 += (y.dim == 3 ? c.mbz : 1))
            for (int y0 = 0; y0 < y.ny; y0 += kMassBY)
                for (int x0 = 0; x0 < y.nx; x0 += kTX) nat.push_back(Tile{s, x0, y0, z0});
        append_xcd_order(nat, c.mtiles);
    }
}

void build_ctiles(apfc_ctx& c) {
    c.ctiles.clear();
    const int H = cheb_halo(c.solver);
    const int IX = kChebShape[c.cheb_shape][0] - 2 * H, IY = kChebShape[c.cheb_shape][1] - 2 * H;
    for (int s = 0; s < c.S; ++s) {
        const Sys& y = c.sys[s];
        std::vector<CTile> nat;
        for (int z = 0; z < y.nz; ++z)
            for (int y0 = 0; y0 < y.ny; y0 += IY)
                for (int x0 = 0; x0 < y.nx; x0 += IX) nat.push_back(CTile{s, x0, y0, z});
        append_xcd_order(nat, c.ctiles);
    }
}

int upload_tables(apfc_ctx& c) {
    HIPCHK(hipMemcpy(c.d_sys, c.sys.data(), sizeof(Sys) * c.S, hipMemcpyHostToDevice));
    for (int l = 0; l < c.mg_n; ++l) {
        HIPCHK(hipMemcpy(c.d_mg_sys[l], c.mg_sys[l].data(), sizeof(Sys) * c.S, hipMemcpyHostToDevice));
        HIPCHK(hipMemcpy(c.d_mg_tiles[l], c.mg_tiles[l].data(), sizeof(Tile) * c.mg_tiles[l].size(),
                         hipMemcpyHostToDevice));
    }
    HIPCHK(hipMemcpy(c.d_tiles, c.tiles.data(), sizeof(Tile) * c.tiles.size(), hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(c.d_chunks, c.chunks.data(), sizeof(Chunk) * c.chunks.size(), hipMemcpyHostToDevice));
    if (!c.ctiles.empty())
        HIPCHK(hipMemcpy(c.d_ctiles, c.ctiles.data(), sizeof(CTile) * c.ctiles.size(), hipMemcpyHostToDevice));
    if (!c.mtiles.empty())
        HIPCHK(hipMemcpy(c.d_mtiles, c.mtiles.data(), sizeof(Tile) * c.mtiles.size(), hipMemcpyHostToDevice));
    return APFC_OK;
}

void invalidate_graphs(apfc_ctx& c) {
    for (auto g : c.graphs)
        if (g) (void)hipGraphExecDestroy(g);
    c.graphs.clear();
    c.graphs_valid = false;
}

// carve the workspace; returns bytes needed (base may be null to only measure)
size_t carve(apfc_ctx& c, char* base) {
    size_t off = 0;
    auto take = [&](size_t bytes) -> char* {
        off = (off + 255) & ~size_t(255);
        char* p = base ? base + off : nullptr;
        off += bytes;
        return p;
    };
    const long long NT = c.NT;
    const int S = c.S, m = c.m;
    const size_t zs = c.zsize();
    c.d_sys = (Sys*)take(sizeof(Sys) * S);
    c.d_tiles = (Tile*)take(sizeof(Tile) * c.max_tiles);
    c.d_chunks = (Chunk*)take(sizeof(Chunk) * c.chunks.size());
    c.d_ctiles = (CTile*)take(sizeof(CTile) * std::max<size_t>(1, c.max_ctiles));
    c.d_mtiles = (Tile*)take(sizeof(Tile) * std::max<size_t>(1, c.mtiles.size()));
    c.d_tab = (double**)take(sizeof(double*) * 4 * c.count);
    c.X = (zd*)take(sizeof(zd) * 2 * NT);
    c.B = (zd*)take(sizeof(zd) * 2 * NT);
    c.R = (zd*)take(sizeof(zd) * 2 * NT);
    c.W = (zd*)take(sizeof(zd) * 2 * NT);
    c.BB = (zd*)take(sizeof(zd) * NT);
    c.V = (zd*)take(sizeof(zd) * 2 * NT * (m + 1));
    c.Z = take(zs * 2 * NT * m);
    for (int i = 0; i < 6; ++i) c.pc[i] = take(zs * NT);
    for (int i = 0; i < 3; ++i) c.hist[i] = i < c.solver.x0_order ? (zd*)take(sizeof(zd) * 2 * NT) : nullptr;
    c.dnode = (double*)take(sizeof(double) * c.NI);
    c.tpart = (double*)take(sizeof(double) * kSlots * c.max_tiles);
    c.cpart = (double*)take(sizeof(double) * (2 * kMaxRestart + 2) * c.chunks.size());
    c.apart = (double*)take(sizeof(double) * (2 * kMaxRestart + 2) * c.max_tiles);
    Krylov& k = c.kr;
    k.m = m;
    k.nv1 = 2 * (m + 1);
    k.rtol = c.solver.rtol;
    k.always_reorth = 0;
    // keep the orthogonality loss of one classical pass (~eps |w|/|w'|) below rtol/100
    {
        const double r = 100.0 * 2.2e-16 / c.solver.rtol;
        k.reorth_theta = std::min(0.5, std::max(1e-6, r * r));
    }
    k.H = (double*)take(sizeof(double) * S * m * 2 * (m + 1));
    k.cs = (double*)take(sizeof(double) * S * m);
    k.sn = (double*)take(sizeof(double) * S * 2 * m);
    k.g = (double*)take(sizeof(double) * S * 2 * (m + 1));
    k.y = (double*)take(sizeof(double) * S * 2 * m);
    k.hsum = (double*)take(sizeof(double) * S * 2 * (m + 1));
    k.hinv = (double*)take(sizeof(double) * S);
    k.red1 = (double*)take(sizeof(double) * S * (k.nv1 + 1));
    k.redr = (double*)take(sizeof(double) * S * kSlots);
    k.bnorm = (double*)take(sizeof(double) * S);
    k.target = (double*)take(sizeof(double) * S);
    k.inv_beta = (double*)take(sizeof(double) * S);
    k.relres = (double*)take(sizeof(double) * S);
    k.solve_active = (int*)take(sizeof(int) * S);
    k.iter_active = (int*)take(sizeof(int) * S);
    k.reorth = (int*)take(sizeof(int) * S);
    k.kcount = (int*)take(sizeof(int) * S);
    k.iters = (int*)take(sizeof(int) * S);
    k.cycles = (int*)take(sizeof(int) * S);
    k.err = (int*)take(sizeof(int) * 4);
    k.tick_c = (int*)take(sizeof(int) * S);
    k.tick_p = (int*)take(sizeof(int));
    c.run_it_sum = (long long*)take(sizeof(long long) * S);
    c.run_it_max = (int*)take(sizeof(int) * S);
    c.run_cyc_max = (int*)take(sizeof(int) * S);
    c.run_res_max = (double*)take(sizeof(double) * S);
    c.pub_dev = (int*)take(sizeof(int) * 8);
    for (int l = 0; l < c.mg_n; ++l) {
        c.d_mg_sys[l] = (Sys*)take(sizeof(Sys) * S);
        c.d_mg_tiles[l] = (Tile*)take(sizeof(Tile) * c.mg_tiles[l].size());
        for (int b = 0; b < 5; ++b) c.mg_buf[l][b] = take(zs * c.mg_NT[l]);
    }
    return off + 256;
}

__global__ void k_reset_counters(Krylov kr, int S) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s < S) {
        kr.iters[s] = 0;
        kr.cycles[s] = 0;
        kr.kcount[s] = 0;
        kr.solve_active[s] = 1;
        kr.iter_active[s] = 0;
        if (s == 0) kr.err[0] = 0;
    }
}

// Statistics of a multi-step run, summed (iterations) or maximised (cycles, residual) over the steps on
// the device, so that the steps need no copies to the host.
__global__ void k_run_stats(Krylov kr, int S, int reset, long long* it_sum, int* it_max, int* cyc_max,
                            double* res_max) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= S) return;
    if (reset) {
        it_sum[s] = 0;
        it_max[s] = 0;
        cyc_max[s] = 0;
        res_max[s] = 0.0;
        return;
    }
    it_sum[s] += kr.iters[s];
    it_max[s] = max(it_max[s], kr.iters[s]);
    cyc_max[s] = max(cyc_max[s], kr.cycles[s]);
    res_max[s] = fmax(res_max[s], kr.relres[s]);
}

int check_mesh(const apfc_mesh& m) {
    if (m.dim != 2 && m.dim != 3) return fail(APFC_ERR_INVALID, "mesh.dim must be 2 or 3");
    const double h = m.length[0] / (double)m.n[0];
    for (int d = 0; d < m.dim; ++d) {
        if (m.n[d] < 4 || m.n[d] > (1 << 20)) return fail(APFC_ERR_INVALID, "mesh.n[d] must be in [4, 2^20]");
        if (!(m.length[d] > 0.0) || !std::isfinite(m.length[d])) return fail(APFC_ERR_INVALID, "mesh.length must be positive");
        const double hd = m.length[d] / (double)m.n[d];
        if (std::fabs(hd - h) > 1e-12 * h) return fail(APFC_ERR_INVALID, "mesh: all directions must share one h");
    }
    return APFC_OK;
}

int check_params(const apfc_params& p) {
    if (!(p.a0 > 0.0) || !std::isfinite(p.a1) || !(p.a2 >= 0.0) || !std::isfinite(p.a2) || !std::isfinite(p.a3))
        return fail(APFC_ERR_INVALID, "params: need a0 > 0, a2 >= 0, finite a1, a3");
    if (p.picard_iters < 1 || p.picard_iters > 100) return fail(APFC_ERR_INVALID, "params.picard_iters must be in [1,100]");
    if (!(p.rtol > 0.0) || p.rtol >= 1.0) return fail(APFC_ERR_INVALID, "params.rtol must be in (0,1)");
    if (p.restart < 1 || p.restart > kMaxRestart) return fail(APFC_ERR_INVALID, "params.restart must be in [1,32]");
    if (p.max_iters < 1) return fail(APFC_ERR_INVALID, "params.max_iters must be >= 1");
    if (p.precision != APFC_FP64 && p.precision != APFC_MIXED) return fail(APFC_ERR_INVALID, "params.precision");
    if (p.mass_iters < 1 || p.mass_iters > kMaxCheb || p.diff_iters < 1 || p.diff_iters > kMaxCheb)
        return fail(APFC_ERR_INVALID, "params: inner iterations must be in [1,64]");
    if (p.inner_kind != APFC_INNER_PCG && p.inner_kind != APFC_INNER_CHEB && p.inner_kind != APFC_INNER_MG)
        return fail(APFC_ERR_INVALID, "params.inner_kind");
    if (p.x0_order < 0 || p.x0_order > 3) return fail(APFC_ERR_INVALID, "params.x0_order must be in [0,3]");
    if (p.mass_kind != APFC_MASS_ITER && p.mass_kind != APFC_MASS_SEPARABLE)
        return fail(APFC_ERR_INVALID, "params.mass_kind");
    if (p.mass_kind == APFC_MASS_SEPARABLE && p.mass_iters > kMassRMax)
        return fail(APFC_ERR_INVALID, "params: APFC_MASS_SEPARABLE takes mass_iters in [1,4] (taps per side)");
    return APFC_OK;
}

int check_lattice(const apfc_lattice& L, int dim) {
    if (L.J < 1 || L.J > kMaxJ) return fail(APFC_ERR_INVALID, "lattice.J must be in [1,8]");
    for (int j = 0; j < L.J; ++j) {
        double n2 = 0.0;
        for (int c = 0; c < 3; ++c) {
            if (!std::isfinite(L.k[j][c])) return fail(APFC_ERR_INVALID, "lattice.k not finite");
            n2 += L.k[j][c] * L.k[j][c];
        }
        if (!(n2 > 0.0)) return fail(APFC_ERR_INVALID, "lattice.k must be nonzero");
        if (dim == 2 && L.k[j][2] != 0.0) return fail(APFC_ERR_INVALID, "lattice: k_z must be 0 in 2D");
    }
    return APFC_OK;
}

}  // namespace

// ----------------------------------------------------------------------------------------------
// public API
// ----------------------------------------------------------------------------------------------
extern "C" {

const char* apfc_last_error(void) { return g_err.c_str(); }

const char* apfc_status_string(int status) {
    switch (status) {
        case APFC_OK: return "ok";
        case APFC_ERR_NOT_CONVERGED: return "FGMRES did not converge within max_iters";
        case APFC_ERR_INVALID: return "invalid argument";
        case APFC_ERR_HIP: return "HIP runtime error";
        case APFC_ERR_WORKSPACE: return "workspace missing or too small";
        case APFC_ERR_NONFINITE: return "non-finite residual";
        default: return "unknown status";
    }
}

void apfc_params_default(apfc_params* p) {
    if (!p) return;
    p->a0 = 0.98;
    p->a1 = 0.01;
    p->a2 = 0.25;
    p->a3 = 0.5;
    p->picard_iters = 1;
    p->rtol = 1e-8;
    p->restart = 30;
    p->max_iters = 500;
    p->precision = APFC_FP64;
    p->mass_iters = 3;
    p->diff_iters = 5;
    p->inner_kind = APFC_INNER_PCG;
    p->x0_order = 0;
    p->mass_kind = APFC_MASS_ITER;
}

int apfc_lattice_default(int kind, apfc_lattice* L) {
    if (!L) return fail(APFC_ERR_INVALID, "lattice is NULL");
    std::memset(L, 0, sizeof(*L));
    L->kind = kind;
    if (kind == APFC_TRI2D) {
        // Eq. (7)
        const double s = std::sqrt(3.0) / 2.0;
        L->J = 3;
        L->k[0][0] = -s; L->k[0][1] = -0.5;
        L->k[1][0] = 0.0; L->k[1][1] = 1.0;
        L->k[2][0] = s; L->k[2][1] = -0.5;
        return APFC_OK;
    }
    if (kind == APFC_BCC3D) {
        const double r = 1.0 / std::sqrt(2.0);
        const double v[6][3] = {{1, 1, 0}, {1, -1, 0}, {1, 0, 1}, {1, 0, -1}, {0, 1, 1}, {0, 1, -1}};
        L->J = 6;
        for (int j = 0; j < 6; ++j)
            for (int c = 0; c < 3; ++c) L->k[j][c] = r * v[j][c];
        return APFC_OK;
    }
    if (kind == APFC_FCC3D) {
        // the first two shells of the fcc reciprocal lattice: <111> (|k| = 1, one of each +- pair, summing
        // to zero) and <200> (|k| = 2/sqrt 3)
        const double r = 1.0 / std::sqrt(3.0);
        const double v[7][3] = {{1, 1, 1}, {1, -1, -1}, {-1, 1, -1}, {-1, -1, 1}, {2, 0, 0}, {0, 2, 0}, {0, 0, 2}};
        L->J = 7;
        for (int j = 0; j < 7; ++j)
            for (int c = 0; c < 3; ++c) L->k[j][c] = r * v[j][c];
        return APFC_OK;
    }
    return fail(APFC_ERR_INVALID, "apfc_lattice_default: kind must be APFC_TRI2D, APFC_BCC3D or APFC_FCC3D");
}

int apfc_uniform_amplitude(const apfc_lattice* L, const apfc_params* p, double* phi) {
    if (!L || !p || !phi) return fail(APFC_ERR_INVALID, "NULL argument");
    if (int rc = check_lattice(*L, 3); rc) return rc;
    Terms T;
    if (int rc = build_terms(*L, T); rc) return rc;
    double c2, c3, c4;
    uniform_poly(T, *p, c2, c3, c4);
    // d f / d phi = phi (2 c2 + 3 c3 phi + 4 c4 phi^2) = 0
    const double disc = 9.0 * c3 * c3 - 32.0 * c2 * c4;
    *phi = (disc < 0.0 || !(c4 > 0.0)) ? 0.0 : (-3.0 * c3 + std::sqrt(disc)) / (8.0 * c4);
    if (*phi < 0.0) *phi = 0.0;
    return APFC_OK;
}

int apfc_equilibrium_amplitudes(const apfc_lattice* L, const apfc_params* p, double* phi) {
    if (!L || !p || !phi) return fail(APFC_ERR_INVALID, "NULL argument");
    double phi0 = 0.0;
    if (int rc = apfc_uniform_amplitude(L, p, &phi0); rc) return rc;
    Terms T;
    if (int rc = build_terms(*L, T); rc) return rc;
    const int J = L->J;
    // shells of equal |k_j|^2
    int shell[kMaxJ], ns = 0;
    double s2[kMaxJ];
    for (int j = 0; j < J; ++j) {
        const double k2 = L->k[j][0] * L->k[j][0] + L->k[j][1] * L->k[j][1] + L->k[j][2] * L->k[j][2];
        int s = 0;
        while (s < ns && std::fabs(s2[s] - k2) > 1e-9 * k2) ++s;
        if (s == ns) s2[ns++] = k2;
        shell[j] = s;
    }
    for (int j = 0; j < J; ++j) phi[j] = phi0;
    if (ns == 1 || phi0 == 0.0) return APFC_OK;
    // d f / d phi_s for real amplitudes eta_j = x[shell(j)]: pair part and the resonant products of T
    auto grad = [&](const double* x, double* g) {
        double e[kMaxJ], A = 0.0;
        for (int j = 0; j < J; ++j) {
            e[j] = x[shell[j]];
            A += 2.0 * e[j] * e[j];
        }
        double gj[kMaxJ];
        for (int j = 0; j < J; ++j)
            gj[j] = p->a1 / p->a0 * 4.0 * e[j] + p->a2 / p->a0 * (8.0 * A * e[j] - 8.0 * e[j] * e[j] * e[j]);
        for (int t = 0; t < T.n; ++t) {
            const double c = T.order[t] == 3 ? -2.0 * p->a3 / p->a0 : 8.0 * p->a2 / p->a0;
            for (int q = 0; q < T.order[t]; ++q) {
                double prod = 2.0 * c;
                for (int r = 0; r < T.order[t]; ++r)
                    if (r != q) prod *= e[T.idx[t][r]];
                gj[T.idx[t][q]] += prod;
            }
        }
        for (int s = 0; s < ns; ++s) g[s] = 0.0;
        for (int j = 0; j < J; ++j) g[shell[j]] += gj[j];
    };
    // Newton's method from the single-shell root, Jacobian by central differences of the gradient
    double x[kMaxJ], g[kMaxJ];
    for (int s = 0; s < ns; ++s) x[s] = phi0;
    for (int it = 0; it < 100; ++it) {
        grad(x, g);
        double gn = 0.0;
        for (int s = 0; s < ns; ++s) gn = std::max(gn, std::fabs(g[s]));
        if (gn < 1e-16) break;
        double Jm[kMaxJ][kMaxJ + 1];
        for (int c = 0; c < ns; ++c) {
            double xp[kMaxJ], xm[kMaxJ], gp[kMaxJ], gm[kMaxJ];
            const double hstep = 1e-6 * phi0;
            for (int s = 0; s < ns; ++s) xp[s] = xm[s] = x[s];
            xp[c] += hstep;
            xm[c] -= hstep;
            grad(xp, gp);
            grad(xm, gm);
            for (int r = 0; r < ns; ++r) Jm[r][c] = (gp[r] - gm[r]) / (2.0 * hstep);
        }
        for (int r = 0; r < ns; ++r) Jm[r][ns] = -g[r];
        // Gaussian elimination with partial pivoting
        for (int c = 0; c < ns; ++c) {
            int piv = c;
            for (int r = c + 1; r < ns; ++r)
                if (std::fabs(Jm[r][c]) > std::fabs(Jm[piv][c])) piv = r;
            for (int q = 0; q <= ns; ++q) std::swap(Jm[c][q], Jm[piv][q]);
            if (Jm[c][c] == 0.0) return fail(APFC_ERR_INVALID, "apfc_equilibrium_amplitudes: singular Newton system");
            for (int r = c + 1; r < ns; ++r) {
                const double f = Jm[r][c] / Jm[c][c];
                for (int q = c; q <= ns; ++q) Jm[r][q] -= f * Jm[c][q];
            }
        }
        double dx[kMaxJ];
        for (int r = ns - 1; r >= 0; --r) {
            double v = Jm[r][ns];
            for (int q = r + 1; q < ns; ++q) v -= Jm[r][q] * dx[q];
            dx[r] = v / Jm[r][r];
        }
        for (int s = 0; s < ns; ++s) x[s] += dx[s];
    }
    for (int s = 0; s < ns; ++s)
        if (!(x[s] > 0.0) || !std::isfinite(x[s]))
            return fail(APFC_ERR_INVALID, "apfc_equilibrium_amplitudes: no crystal with all amplitudes positive");
    for (int j = 0; j < J; ++j) phi[j] = x[shell[j]];
    return APFC_OK;
}

int apfc_create_batch(int count, const apfc_mesh* meshes, const apfc_lattice* lattice, const apfc_params* params,
                      apfc_ctx** out) {
    if (!out) return fail(APFC_ERR_INVALID, "out is NULL");
    *out = nullptr;
    if (count < 1 || count > 4096 || !meshes || !lattice || !params)
        return fail(APFC_ERR_INVALID, "apfc_create_batch: need 1 <= count <= 4096 and non-NULL arrays");
    const int dim = meshes[0].dim;
    for (int b = 0; b < count; ++b) {
        if (int rc = check_mesh(meshes[b]); rc) return rc;
        if (meshes[b].dim != dim) return fail(APFC_ERR_INVALID, "all instances must have the same dim");
        if (int rc = check_params(params[b]); rc) return rc;
        const apfc_params& a = params[0];
        const apfc_params& p = params[b];
        if (p.picard_iters != a.picard_iters || p.rtol != a.rtol || p.restart != a.restart ||
            p.max_iters != a.max_iters || p.precision != a.precision || p.mass_iters != a.mass_iters ||
            p.diff_iters != a.diff_iters || p.inner_kind != a.inner_kind || p.x0_order != a.x0_order)
            return fail(APFC_ERR_INVALID, "solver fields of params[] must be equal across instances");
    }
    if (int rc = check_lattice(*lattice, dim); rc) return rc;
    auto c = new apfc_ctx();
    c->count = count;
    c->J = lattice->J;
    c->dim = dim;
    c->lattice = *lattice;
    c->meshes.assign(meshes, meshes + count);
    c->params.assign(params, params + count);
    c->solver = params[0];
    c->m = params[0].restart;
    c->mixed = params[0].precision == APFC_MIXED;
    if (int rc = build_terms(*lattice, c->terms); rc) {
        delete c;
        return rc;
    }
    if (params[0].inner_kind == APFC_INNER_CHEB) {
        if (dim == 2 && cheb_halo(params[0]) > 12) {
            delete c;
            return fail(APFC_ERR_INVALID, "APFC_INNER_CHEB needs mass_iters <= 13 and diff_iters <= 12");
        }
        if (dim == 2 && cheb_halo(params[0]) > 8) {
            // the smaller region shapes need interior tiles of at least 16 x 16
            delete c;
            return fail(APFC_ERR_INVALID, "APFC_INNER_CHEB in 2D needs mass_iters <= 9 and diff_iters <= 8");
        }
    }
    c->S = count * c->J;
    long long off = 0, doff = 0;
    for (int b = 0; b < count; ++b) {
        const apfc_mesh& m = meshes[b];
        const long long nx = m.n[0], ny = m.n[1], nz = dim == 3 ? m.n[2] : 1;
        const long long N = nx * ny * nz;
        const double h = m.length[0] / (double)nx;
        for (int j = 0; j < c->J; ++j) {
            Sys y{};
            y.inst = b;
            y.j = j;
            y.dim = dim;
            y.nx = (int)nx;
            y.ny = (int)ny;
            y.nz = (int)nz;
            y.N = N;
            y.off = off;
            y.doff = doff;
            y.h = h;
            y.w = std::pow(h, dim);
            set_wsep(y);
            double k2 = 0.0;
            for (int q = 0; q < 3; ++q) {
                y.kv[q] = lattice->k[j][q];
                k2 += y.kv[q] * y.kv[q];
            }
            y.kappa = params[b].a0 * k2;      // kappa_j = a0 |k_j|^2 (below Eq. (3))
            y.a0 = params[b].a0;
            y.a1 = params[b].a1;
            y.a2 = params[b].a2;
            y.a3 = params[b].a3;
            // Jacobi diagonals: M_ii = (2h/3)^dim, K_ii = dim (2/h) (2h/3)^(dim-1)
            y.diagM = std::pow(2.0 * h / 3.0, dim);
            y.diagK = dim * (2.0 / h) * std::pow(2.0 * h / 3.0, dim - 1);
            c->sys.push_back(y);
            off += N;
        }
        doff += N;
    }
    c->NT = off;
    c->NI = doff;
    for (int s = 0; s < c->S; ++s) {
        Sys& y = c->sys[s];
        y.cbeg = (int)c->chunks.size();
        for (long long e0 = 0; e0 < 2 * y.N; e0 += kChunk) c->chunks.push_back(Chunk{s, (int)e0});
        y.cend = (int)c->chunks.size();
    }
    if (params[0].inner_kind == APFC_INNER_MG) {
        if (int rc = build_mg_levels(*c); rc) {
            delete c;
            return rc;
        }
    }
    build_mtiles(*c);
    std::vector<Tile> t4;
    build_tiles(*c, 4, t4);
    c->max_tiles = (int)t4.size();
    c->TY = 16;
    build_tiles(*c, c->TY, c->tiles);
    set_dt_scalars(*c, 1.0);
    if (params[0].inner_kind == APFC_INNER_CHEB && dim == 2) {
        for (int sh = 0; sh < kChebShapes; ++sh) {
            c->cheb_shape = sh;
            build_ctiles(*c);
            c->max_ctiles = std::max(c->max_ctiles, c->ctiles.size());
        }
        c->cheb_shape = 0;
        build_ctiles(*c);
    }
    {
        apfc_ctx tmp_view = *c;      // sizes only: carve on a copy
        c->ws_need = carve(tmp_view, nullptr);
    }
    c->na_ptrs.assign(4 * (size_t)count, nullptr);
    c->na_tab.assign(4 * (size_t)count, nullptr);
    c->na_flags.assign(2 * (size_t)c->S + 8, 0);
    c->na_dbl.assign((size_t)c->S + 8, 0.0);
    c->tab_shadow.reserve(4 * (size_t)count);
    *out = c;
    return APFC_OK;
}

int apfc_create(const apfc_mesh* mesh, const apfc_lattice* lattice, const apfc_params* params, apfc_ctx** out) {
    return apfc_create_batch(1, mesh, lattice, params, out);
}

size_t apfc_workspace_bytes(const apfc_ctx* c) { return c ? c->ws_need : 0; }

int apfc_set_workspace(apfc_ctx* c, void* ptr, size_t bytes) {
    if (!c || !ptr) return fail(APFC_ERR_INVALID, "NULL argument");
    if (((uintptr_t)ptr & 255) != 0) return fail(APFC_ERR_WORKSPACE, "workspace must be 256-byte aligned");
    if (bytes < apfc_workspace_bytes(c)) return fail(APFC_ERR_WORKSPACE, "workspace smaller than apfc_workspace_bytes");
    invalidate_graphs(*c);
    if (!c->h_tab) {
        // pinned host staging for pointer tables and flag / scalar read-back
        if (hipHostMalloc((void**)&c->h_tab, sizeof(double*) * 4 * c->count) != hipSuccess ||
            hipHostMalloc((void**)&c->h_flags, sizeof(int) * (4 * c->S + 8)) != hipSuccess ||
            hipHostMalloc((void**)&c->h_dbl, sizeof(double) * (kSlots * c->S + 8)) != hipSuccess ||
            hipHostMalloc((void**)&c->h_pub, sizeof(int) * 8, hipHostMallocMapped | hipHostMallocCoherent) != hipSuccess)
            return fail(APFC_ERR_HIP, "hipHostMalloc of host staging buffers failed");
        HIPCHK(hipHostGetDevicePointer((void**)&c->d_pub, c->h_pub, 0));
    }
    c->ws = (char*)ptr;
    c->ws_bytes = bytes;
    c->ws_user = c->ws;
    c->ws_user_bytes = bytes;
    c->hist_n = 0;
    c->tab_shadow.clear();
    carve(*c, c->ws);
    // the tickets of the fused second-pass reduction start at zero; every launch leaves them at zero
    HIPCHK(hipMemset(c->kr.tick_c, 0, sizeof(int) * c->S));
    HIPCHK(hipMemset(c->kr.tick_p, 0, sizeof(int)));
    return upload_tables(*c);
}

int apfc_destroy(apfc_ctx* c) {
    if (!c) return APFC_OK;
    noalloc_forget(c);
    invalidate_graphs(*c);
    if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
    if (c->probe.created) {
        for (auto& e : c->probe.ev) (void)hipEventDestroy(e);
        (void)hipFree(c->probe.d_frac);
    }
    if (c->h_tab) (void)hipHostFree(c->h_tab);
    if (c->h_flags) (void)hipHostFree(c->h_flags);
    if (c->h_pub) (void)hipHostFree(c->h_pub);
    if (c->h_dbl) (void)hipHostFree(c->h_dbl);
    delete c;
    return APFC_OK;
}

}  // extern "C"

// ----------------------------------------------------------------------------------------------
// the solver
// ----------------------------------------------------------------------------------------------
namespace {

int need_ws(apfc_ctx* c) {
    if (!c) return fail(APFC_ERR_INVALID, "ctx is NULL");
    if (!c->ws_user) return fail(APFC_ERR_WORKSPACE, "no workspace attached (apfc_set_workspace)");
    if (c->ws != c->ws_user) {
        // the last call ran on the static scratch (apfc_step_noalloc): back onto the caller's workspace,
        // whose tables were left as they were; the states kept for the initial guess were in the scratch
        c->ws = c->ws_user;
        c->ws_bytes = c->ws_user_bytes;
        carve(*c, c->ws);
        c->hist_n = 0;
        c->tab_shadow.clear();
        invalidate_graphs(*c);
    }
    return APFC_OK;
}

int refresh_dt(apfc_ctx* c, double dt, hipStream_t st) {
    if (!(dt > 0.0) || !std::isfinite(dt)) return fail(APFC_ERR_INVALID, "dt must be positive and finite");
    if (dt != c->dt) {
        set_dt_scalars(*c, dt);
        HIPCHK(hipMemcpyAsync(c->d_sys, c->sys.data(), sizeof(Sys) * c->S, hipMemcpyHostToDevice, st));
        // the multigrid levels' dt scalars and smoothing tables as well
        for (int l = 0; l < c->mg_n; ++l)
            HIPCHK(hipMemcpyAsync(c->d_mg_sys[l], c->mg_sys[l].data(), sizeof(Sys) * c->S, hipMemcpyHostToDevice, st));
        HIPCHK(hipStreamSynchronize(st));
    }
    return APFC_OK;
}

// upload up to 4 tables of per-instance device pointers
int upload_ptrs(apfc_ctx* c, const std::vector<const void*>* tabs, int ntabs, hipStream_t st) {
    if (c->noalloc) return fail(APFC_ERR_INVALID, "internal: pointer tables of a no-alloc call go through upload_ptrs_na");
    std::vector<const void*> flat;
    for (int t = 0; t < ntabs; ++t) flat.insert(flat.end(), tabs[t].begin(), tabs[t].end());
    if (flat.size() <= c->tab_shadow.size() && std::equal(flat.begin(), flat.end(), c->tab_shadow.begin()))
        return APFC_OK;   // the device tables already hold these pointers
    // the pinned staging buffer may still feed an earlier copy
    HIPCHK(hipStreamSynchronize(st));
    for (size_t i = 0; i < flat.size(); ++i) c->h_tab[i] = (double*)flat[i];
    HIPCHK(hipMemcpyAsync(c->d_tab, c->h_tab, sizeof(double*) * flat.size(), hipMemcpyHostToDevice, st));
    c->tab_shadow = flat;
    return APFC_OK;
}
double* const* tab(apfc_ctx* c, int t) { return c->d_tab + t * c->count; }

// upload_ptrs for apfc_step_noalloc: the n pointers staged in c->na_ptrs go through the pageable
// c->na_tab (sized at create) with a synchronous copy; nothing is allocated.
int upload_ptrs_na(apfc_ctx* c, int n, hipStream_t st) {
    HIPCHK(hipStreamSynchronize(st));
    for (int i = 0; i < n; ++i) c->na_tab[i] = (double*)c->na_ptrs[i];
    HIPCHK(hipMemcpyAsync(c->d_tab, c->na_tab.data(), sizeof(double*) * n, hipMemcpyHostToDevice, st));
    HIPCHK(hipStreamSynchronize(st));
    c->tab_shadow.clear();
    return APFC_OK;
}

// Where k_cycle_start publishes the host summary: mapped pinned host memory, or in a no-alloc call a
// device slot copied to the host after the cycle.
int* pub_target(apfc_ctx* c) { return c->noalloc ? c->pub_dev : c->d_pub; }

// The multigrid levels' device view (tables and buffers of the attached workspace).
MgLevels mg_levels(apfc_ctx* c, const Dev& fine) {
    MgLevels m;
    m.n = c->mg_n;
    m.nu = c->solver.diff_iters;
    m.coarse_its = 24;
    for (int l = 0; l < c->mg_n; ++l) {
        Dev d = fine;
        d.sys = c->d_mg_sys[l];
        d.tiles = c->d_mg_tiles[l];
        d.ntiles = (int)c->mg_tiles[l].size();
        d.TY = 16;
        d.NT = c->mg_NT[l];
        m.lev[l] = d;
        m.x[l] = c->mg_buf[l][0];
        m.b[l] = c->mg_buf[l][1];
        m.r[l] = c->mg_buf[l][2];
        m.d0[l] = c->mg_buf[l][3];
        m.d1[l] = c->mg_buf[l][4];
    }
    return m;
}

// P^{-1} v -> z with the context's inner solver: fused 2D Chebyshev tiles, one-launch-per-iteration
// Chebyshev (3D), or the paper's Jacobi-PCG.  With vin.src set (fused 2D Chebyshev only), v is formed
// from vin and stored to vin.vout.
template <typename T>
void precond(apfc_ctx* c, const Dev& d, const cx<T>* v, cx<T>* z, const int* mask, hipStream_t st,
             const VIn<T>& vin = VIn<T>{}) {
    cx<T>** pc = (cx<T>**)c->pc;
    const int sep = c->solver.mass_kind == APFC_MASS_SEPARABLE ? c->solver.mass_iters : 0;
    if (c->solver.inner_kind == APFC_INNER_MG)
        launch_precond_mg<T>(d, mg_levels(c, d), v, z, pc[0], pc[1], pc[2], pc[3], pc[4], pc[5],
                             c->solver.mass_iters, sep, mask, st);
    else if (c->solver.inner_kind == APFC_INNER_CHEB && c->dim == 2)
        launch_precond_cheb<T>(d, c->cheb_shape, c->d_ctiles, (int)c->ctiles.size(), cheb_halo(c->solver), v, z,
                               pc[0], pc[1], c->solver.mass_iters, c->solver.diff_iters, sep, vin, mask, st);
    else if (c->solver.inner_kind == APFC_INNER_CHEB)
        launch_precond_cheb_unfused<T>(d, v, z, pc[0], pc[1], pc[2], pc[3], pc[4], c->solver.mass_iters,
                                       c->solver.diff_iters, sep, mask, st);
    else
        launch_precond<T>(d, v, z, pc[0], pc[1], pc[2], pc[3], pc[4], pc[5], c->tpart, c->solver.mass_iters,
                          c->solver.diff_iters, sep, mask, st);
}

// The fused 2D Chebyshev preconditioner forms the basis vectors itself: the first of a cycle from the
// residual (no separate scaling pass), the others from w and the earlier ones (no projection pass).
bool precond_forms_basis(const apfc_ctx* c) { return c->solver.inner_kind == APFC_INNER_CHEB && c->dim == 2; }

// The Krylov basis V is stored in the preconditioner's precision T: FP32 in mixed precision (inner
// products and projections still accumulate in FP64), FP64 otherwise.
template <typename T>
cx<T>* basis(apfc_ctx* c) { return (cx<T>*)c->V; }
// The restart residual r = b - A x is stored in the same precision: only v_0 = r / |r| is formed from
// it (its norm is reduced from the FP64 values).
template <typename T>
cx<T>* residual(apfc_ctx* c) { return (cx<T>*)c->R; }
void launch_restart_residual(apfc_ctx* c, const Dev& d, const int* mask, hipStream_t st) {
    if (c->mixed)
        launch_residual<zf>(d, c->X, c->B, c->dnode, residual<float>(c), c->tpart, mask, st);
    else
        launch_residual<zd>(d, c->X, c->B, c->dnode, residual<double>(c), c->tpart, mask, st);
}

// v_0 = r / beta where the preconditioner does not form it
void scale_start(apfc_ctx* c, const Dev& d, hipStream_t st) {
    if (precond_forms_basis(c)) return;
    if (c->mixed)
        launch_scale<zf>(d, residual<float>(c), c->kr.inv_beta, basis<float>(c), c->kr.iter_active, st);
    else
        launch_scale<zd>(d, residual<double>(c), c->kr.inv_beta, basis<double>(c), c->kr.iter_active, st);
}

template <typename T>
void iteration(apfc_ctx* c, const Dev& d, int k, hipStream_t st) {
    const Krylov& kr = c->kr;
    const long long vs = c->vstride();
    cx<T>* Z = (cx<T>*)c->Z;
    cx<T>* V = basis<T>(c);
    const int* act = kr.iter_active;
    // w is kept in the basis precision (the front of the W buffer)
    cx<T>* Wk = (cx<T>*)c->W;
    const bool form_v = precond_forms_basis(c);
    if (form_v) {
        // the preconditioner's first stages form v_k and store it: v_0 = r / beta, or
        // v_k = (w_{k-1} - sum_{l < k} h_{l,k-1} v_l) / h_{k,k-1} with the previous iteration's column
        VIn<T> vin;
        vin.vout = V + k * vs;
        if (k == 0) {
            vin.src = residual<T>(c);
            vin.scale = kr.inv_beta;
        } else {
            vin.src = Wk;
            vin.V = V;
            vin.vs = vs;
            vin.nv = k;
            vin.hcoef = kr.hsum;
            vin.hld = 2 * (c->m + 1);
            vin.scale = kr.hinv;
        }
        precond<T>(c, d, nullptr, Z + k * vs, act, st, vin);
    } else {
        precond<T>(c, d, V + k * vs, Z + k * vs, act, st);
    }
    const int nv = k + 1;
    // W = A z_k with the first Gram-Schmidt pass fused (V^H w and |w|^2 per tile)
    launch_apply_dot<T>(d, Z + k * vs, c->dnode, Wk, V, vs, nv, c->apart, act, st);
    // reduce the first pass; skip or run the second; Hessenberg column, Givens, convergence test
    launch_gs<cx<T>>(d, kr, k, c->apart, V, vs, Wk, c->cpart, st);
    // v_{k+1}, unless the next preconditioner forms it; the cycle's last one, v_m, is not needed: the
    // solution update reads Z, and the next cycle starts from the recomputed residual
    if (k + 1 < c->m && !form_v)
        launch_proj_final<cx<T>>(d, V, vs, nv, Wk, kr.hsum, kr.hinv, 2 * (c->m + 1), V + (k + 1) * vs, act, st);
}

void run_iteration(apfc_ctx* c, const Dev& d, int k, hipStream_t st) {
    if (c->mixed)
        iteration<float>(c, d, k, st);
    else
        iteration<double>(c, d, k, st);
}

// One restart cycle: m Arnoldi iterations (masked per system once it has converged or broken
// down), the solution update, the true FP64 residual, the next cycle's start vector and the
// published flags.
void run_cycle(apfc_ctx* c, const Dev& d, hipStream_t st) {
    Krylov& kr = c->kr;
    const long long vs = c->vstride();
    for (int k = 0; k < c->m; ++k) run_iteration(c, d, k, st);
    launch_solve_y(d, kr, st);
    if (c->mixed)
        launch_xupdate<float>(d, (const zf*)c->Z, vs, kr.kcount, kr.y, 2 * c->m, c->X, kr.solve_active, st);
    else
        launch_xupdate<double>(d, (const zd*)c->Z, vs, kr.kcount, kr.y, 2 * c->m, c->X, kr.solve_active, st);
    launch_restart_residual(c, d, kr.solve_active, st);
    launch_cycle_start(d, kr, c->tpart, false, pub_target(c), st);
    scale_start(c, d, st);
}

int capture_graphs(apfc_ctx* c) {
    if (!c->cap_stream) HIPCHK(hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking));
    invalidate_graphs(*c);
    Dev d = c->dev();
    d.probe = nullptr;
    c->graphs.assign(1, nullptr);
    hipGraph_t g;
    HIPCHK(hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal));
    run_cycle(c, d, c->cap_stream);
    HIPCHK(hipStreamEndCapture(c->cap_stream, &g));
    hipGraphExec_t ge;
    hipError_t e = hipGraphInstantiate(&ge, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) return fail(APFC_ERR_HIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
    c->graphs[0] = ge;
    c->graphs_valid = true;
    return APFC_OK;
}

// Host wait for the end of a restart cycle.  The convergence check sits on the critical path of every
// time step, and a blocking wait adds the wake-up latency of the waiting thread (tens of microseconds)
// to each step, so the host polls the stream instead.
hipError_t poll_sync(hipStream_t st) {
    for (;;) {
        const hipError_t e = hipStreamQuery(st);
        if (e != hipErrorNotReady) return e;
    }
}

// Restarted FGMRES on every system: B and the initial guess X must be set, dnode current.
int fgmres(apfc_ctx* c, hipStream_t st, int* total_iters) {
    Dev d = c->dev();
    Krylov& kr = c->kr;
    const long long vs = c->vstride();
    const bool graphs = c->use_graphs && d.probe == nullptr && !c->noalloc;
    if (graphs && !c->graphs_valid)
        if (int rc = capture_graphs(c); rc) return rc;
    hipLaunchKernelGGL(k_reset_counters, dim3((c->S + 63) / 64), dim3(64), 0, st, kr, c->S);
    launch_restart_residual(c, d, nullptr, st);
    launch_cycle_start(d, kr, c->tpart, true, nullptr, st);
    scale_start(c, d, st);
    int launched = 0;
    // Cycles before the last one of the previous solve are queued without a host round trip:
    // the iteration count changes slowly from step to step, and a cycle queued for systems that
    // have converged only runs masked (empty) kernels.
    const int hint = c->cycle_hint;
    for (int cyc = 0;; ++cyc) {
        if (graphs)
            HIPCHK(hipGraphLaunch(c->graphs[0], st));
        else
            run_cycle(c, d, st);
        launched += c->m;
        if (cyc + 1 < hint) continue;
        HIPCHK(poll_sync(st));
        // k_cycle_start wrote: [0] any system still solving, [1] non-finite residual, [2] largest iteration count
        const volatile int* pub = c->h_pub;
        if (c->noalloc) {
            HIPCHK(hipMemcpyAsync(c->na_pub, c->pub_dev, sizeof(int) * 3, hipMemcpyDeviceToHost, st));
            HIPCHK(hipStreamSynchronize(st));
            pub = c->na_pub;
        }
        if (pub[1]) return fail(APFC_ERR_NONFINITE, "non-finite residual in FGMRES");
        if (!pub[0]) {
            launched = pub[2];
            break;
        }
        if (pub[2] >= c->solver.max_iters) {
            if (total_iters) *total_iters = pub[2];
            return fail(APFC_ERR_NOT_CONVERGED, "FGMRES reached max_iters");
        }
    }
    if (total_iters) *total_iters = launched;
    c->cycle_hint = (launched + c->m - 1) / c->m;
    return APFC_OK;
}

int fill_stats(apfc_ctx* c, hipStream_t st, apfc_stats* stats, double ms) {
    if (!stats) return APFC_OK;
    const int S = c->S;
    int* flags = c->noalloc ? c->na_flags.data() : c->h_flags;
    double* dbl = c->noalloc ? c->na_dbl.data() : c->h_dbl;
    HIPCHK(hipMemcpyAsync(flags, c->kr.iters, sizeof(int) * S, hipMemcpyDeviceToHost, st));
    HIPCHK(hipMemcpyAsync(flags + S, c->kr.cycles, sizeof(int) * S, hipMemcpyDeviceToHost, st));
    HIPCHK(hipMemcpyAsync(dbl, c->kr.relres, sizeof(double) * S, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    stats->total_iters = 0;
    stats->max_iters = 0;
    stats->cycles = 0;
    stats->max_relres = 0.0;
    for (int s = 0; s < S; ++s) {
        stats->total_iters += flags[s];
        stats->max_iters = std::max(stats->max_iters, flags[s]);
        stats->cycles = std::max(stats->cycles, flags[S + s]);
        stats->max_relres = std::max(stats->max_relres, dbl[s]);
        if (stats->iters) stats->iters[s] = flags[s];
    }
    stats->ms = ms;
    return APFC_OK;
}

int check_states(apfc_ctx* c, const apfc_state* states, bool need_zeta) {
    if (!states) return fail(APFC_ERR_INVALID, "states is NULL");
    for (int b = 0; b < c->count; ++b)
        if (!states[b].eta || (need_zeta && !states[b].zeta)) return fail(APFC_ERR_INVALID, "state pointer is NULL");
    return APFC_OK;
}

}  // namespace

extern "C" {

namespace {

// One step of Algorithm 1 on the state held in X (zeta half, eta half): RHS, K Picard iterates with the
// nodal linearisation, FGMRES.  *max_iters receives the largest per-system iteration count.
int step_body(apfc_ctx* c, const Dev& d, double dt, bool source, hipStream_t st, int* max_iters) {
    const int K = c->solver.picard_iters;
    // 2D with one linearisation: the RHS and the nonlinearity in one pass; 3D: the mass term by the plane
    // march into BB, then the nodal pass (a 27-point stencil per amplitude from global loads costs more
    // than the extra pass over BB)
    const bool fused_rhs = K == 1 && c->dim == 2;
    if (fused_rhs)
        launch_rhs_nonlinear(d, c->X + c->NT, source ? tab(c, 2) : nullptr, c->dnode, c->B, st);
    else
        launch_rhs_base(d, c->X + c->NT, source ? tab(c, 2) : nullptr, c->BB, st);
    const int order = c->solver.x0_order;
    if (order > 0 && c->hist_n > 0 && dt != c->hist_dt) c->hist_n = 0;
    for (int k = 0; k < K; ++k) {
        // all amplitudes linearised at the previous iterate (Jacobi splitting)
        if (!fused_rhs) launch_nonlinear(d, c->X + c->NT, c->BB, c->dnode, c->B, st);
        if (k == 0 && order > 0) {
            // initial guess extrapolated from the kept states; the state passed in becomes the newest
            // kept state and the oldest one is dropped
            const int Q = order, use = std::min(order, c->hist_n);
            const zd* h[3] = {nullptr, nullptr, nullptr};
            for (int q = 0; q < use; ++q) h[q] = c->hist[(c->hist_newest - q + Q) % Q];
            const int oldest = (c->hist_newest + 1) % Q;
            if (!c->use_graphs || c->noalloc) {
                // the guess goes to the scratch buffer W, which then becomes X; the state's buffer is
                // kept as it is as the newest state, and the dropped state's buffer becomes W
                launch_extrapolate(d, c->X, h, c->W, nullptr, use, st);
                zd* state = c->X;
                c->X = c->W;
                c->W = c->hist[oldest];
                c->hist[oldest] = state;
                // captured cycles held X's old address (a no-alloc call frees nothing: it only marks them)
                if (c->noalloc) c->graphs_valid = false;
                else invalidate_graphs(*c);
            } else {
                // captured cycles hold X's address: copy the state, extrapolate in place
                launch_extrapolate(d, c->X, h, c->X, c->hist[oldest], use, st);
            }
            c->hist_newest = oldest;
            c->hist_n = std::min(c->hist_n + 1, Q);
            c->hist_dt = dt;
        }
        if (int rc = fgmres(c, st, max_iters); rc) {
            c->hist_n = 0;
            return rc;
        }
    }
    return APFC_OK;
}

int prepare_step(apfc_ctx* c, apfc_state* states, double dt, const double* const* source, hipStream_t st) {
    if (int rc = need_ws(c); rc) return rc;
    if (int rc = check_states(c, states, true); rc) return rc;
    if (int rc = refresh_dt(c, dt, st); rc) return rc;
    std::vector<const void*> t[3];
    for (int b = 0; b < c->count; ++b) {
        t[0].push_back(states[b].eta);
        t[1].push_back(states[b].zeta);
        t[2].push_back(source ? source[b] : nullptr);
        if (source && !source[b]) return fail(APFC_ERR_INVALID, "source[b] is NULL");
    }
    return upload_ptrs(c, t, 3, st);
}

}  // namespace

int apfc_step(apfc_ctx* c, apfc_state* states, double dt, const double* const* source, void* stream,
              apfc_stats* stats) {
    auto t0 = std::chrono::steady_clock::now();
    hipStream_t st = (hipStream_t)stream;
    if (int rc = prepare_step(c, states, dt, source, st); rc) return rc;
    Dev d = c->dev();
    launch_state_in(d, tab(c, 0), tab(c, 1), c->X, st);
    int iters = 0;
    if (int rc = step_body(c, d, dt, source != nullptr, st, &iters); rc) {
        (void)fill_stats(c, st, stats, 0.0);
        return rc;
    }
    launch_state_out(d, c->X, tab(c, 0), tab(c, 1), st);
    HIPCHK(hipGetLastError());
    const double ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    return fill_stats(c, st, stats, ms);
}

int apfc_run(apfc_ctx* c, apfc_state* states, double dt, int nsteps, const double* const* source, void* stream,
             apfc_stats* stats, int* step_max_iters) {
    auto t0 = std::chrono::steady_clock::now();
    if (nsteps < 1) return fail(APFC_ERR_INVALID, "nsteps must be >= 1");
    hipStream_t st = (hipStream_t)stream;
    if (int rc = prepare_step(c, states, dt, source, st); rc) return rc;
    Dev d = c->dev();
    const int S = c->S;
    const dim3 sg((S + 63) / 64), sb(64);
    hipLaunchKernelGGL(k_run_stats, sg, sb, 0, st, c->kr, S, 1, c->run_it_sum, c->run_it_max, c->run_cyc_max,
                       c->run_res_max);
    launch_state_in(d, tab(c, 0), tab(c, 1), c->X, st);
    int rc = APFC_OK;
    for (int m = 0; m < nsteps && rc == APFC_OK; ++m) {
        int iters = 0;
        rc = step_body(c, d, dt, source != nullptr, st, &iters);
        if (step_max_iters) step_max_iters[m] = iters;
        if (rc == APFC_OK || rc == APFC_ERR_NOT_CONVERGED)
            hipLaunchKernelGGL(k_run_stats, sg, sb, 0, st, c->kr, S, 0, c->run_it_sum, c->run_it_max,
                               c->run_cyc_max, c->run_res_max);
    }
    if (rc == APFC_OK) launch_state_out(d, c->X, tab(c, 0), tab(c, 1), st);
    HIPCHK(hipGetLastError());
    if (stats) {
        std::vector<long long> it_sum(S);
        std::vector<int> it_max(S), cyc_max(S);
        std::vector<double> res_max(S);
        HIPCHK(hipMemcpyAsync(it_sum.data(), c->run_it_sum, sizeof(long long) * S, hipMemcpyDeviceToHost, st));
        HIPCHK(hipMemcpyAsync(it_max.data(), c->run_it_max, sizeof(int) * S, hipMemcpyDeviceToHost, st));
        HIPCHK(hipMemcpyAsync(cyc_max.data(), c->run_cyc_max, sizeof(int) * S, hipMemcpyDeviceToHost, st));
        HIPCHK(hipMemcpyAsync(res_max.data(), c->run_res_max, sizeof(double) * S, hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
        long long total = 0;
        stats->max_iters = 0;
        stats->cycles = 0;
        stats->max_relres = 0.0;
        for (int s = 0; s < S; ++s) {
            total += it_sum[s];
            if (stats->iters) stats->iters[s] = (int)std::min<long long>(it_sum[s], INT32_MAX);
            stats->max_iters = std::max(stats->max_iters, it_max[s]);
            stats->cycles = std::max(stats->cycles, cyc_max[s]);
            stats->max_relres = std::max(stats->max_relres, res_max[s]);
        }
        stats->total_iters = (int)std::min<long long>(total, INT32_MAX);
        stats->ms = rc == APFC_OK
                        ? std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count()
                        : 0.0;
    }
    return rc;
}

int apfc_reset_history(apfc_ctx* c) {
    if (!c) return fail(APFC_ERR_INVALID, "ctx is NULL");
    c->hist_n = 0;
    return APFC_OK;
}

int apfc_init_zeta(apfc_ctx* c, apfc_state* states, void* stream) {
    if (int rc = need_ws(c); rc) return rc;
    if (int rc = check_states(c, states, true); rc) return rc;
    c->hist_n = 0;
    hipStream_t st = (hipStream_t)stream;
    std::vector<const void*> t[2];
    for (int b = 0; b < c->count; ++b) {
        t[0].push_back(states[b].eta);
        t[1].push_back(states[b].zeta);
    }
    if (int rc = upload_ptrs(c, t, 2, st); rc) return rc;
    Dev d = c->dev();
    d.probe = nullptr;
    launch_state_in(d, tab(c, 0), nullptr, c->X, st);
    const int it = c->dim == 2 ? 60 : 100;
    launch_mass_solve(d, c->X + c->NT, c->R, c->R + c->NT, c->W, c->W + c->NT, c->B, c->tpart, it, st);
    launch_planar_out(d, c->R, tab(c, 1), st);
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(st));
    return APFC_OK;
}

int apfc_energy(apfc_ctx* c, const apfc_state* states, double* host_out, void* stream) {
    if (int rc = need_ws(c); rc) return rc;
    if (int rc = check_states(c, states, false); rc) return rc;
    if (!host_out) return fail(APFC_ERR_INVALID, "host_out is NULL");
    hipStream_t st = (hipStream_t)stream;
    std::vector<const void*> t[1];
    for (int b = 0; b < c->count; ++b) t[0].push_back(states[b].eta);
    if (int rc = upload_ptrs(c, t, 1, st); rc) return rc;
    Dev d = c->dev();
    d.probe = nullptr;
    launch_state_in(d, tab(c, 0), nullptr, c->X, st);
    const int it = c->dim == 2 ? 60 : 100;
    launch_mass_solve(d, c->X + c->NT, c->R, c->R + c->NT, c->W, c->W + c->NT, c->B, c->tpart, it, st);
    launch_energy_parts(d, c->X + c->NT, c->R, c->tpart, st);
    launch_reduce(d, c->tpart, kE0, 2, false, c->kr.redr, kSlots, nullptr, st);
    HIPCHK(hipMemcpyAsync(c->h_dbl, c->kr.redr, sizeof(double) * kSlots * c->S, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    for (int b = 0; b < c->count; ++b) {
        double e = 0.0;
        for (int j = 0; j < c->J; ++j) e += c->h_dbl[(b * c->J + j) * kSlots + 0];
        e += c->h_dbl[(b * c->J) * kSlots + 1];
        host_out[b] = e;
    }
    return APFC_OK;
}

int apfc_energy_grad(apfc_ctx* c, const apfc_state* states, double* const* grad, double* ddB, void* stream) {
    if (int rc = need_ws(c); rc) return rc;
    if (int rc = check_states(c, states, false); rc) return rc;
    if (!grad) return fail(APFC_ERR_INVALID, "grad is NULL");
    hipStream_t st = (hipStream_t)stream;
    std::vector<const void*> t[2];
    for (int b = 0; b < c->count; ++b) {
        if (!grad[b]) return fail(APFC_ERR_INVALID, "grad[b] is NULL");
        t[0].push_back(states[b].eta);
        t[1].push_back(grad[b]);
    }
    if (int rc = upload_ptrs(c, t, 2, st); rc) return rc;
    Dev d = c->dev();
    d.probe = nullptr;
    launch_state_in(d, tab(c, 0), nullptr, c->X, st);
    const int it = c->dim == 2 ? 60 : 100;
    launch_mass_solve(d, c->X + c->NT, c->R, c->R + c->NT, c->W, c->W + c->NT, c->B, c->tpart, it, st);
    launch_energy_grad(d, c->X + c->NT, c->R, tab(c, 1), c->tpart, st);
    launch_reduce(d, c->tpart, kE1, 1, false, c->kr.redr, kSlots, nullptr, st);
    HIPCHK(hipMemcpyAsync(c->h_dbl, c->kr.redr, sizeof(double) * kSlots * c->S, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    if (ddB)
        for (int b = 0; b < c->count; ++b) ddB[b] += c->h_dbl[(b * c->J) * kSlots];
    return APFC_OK;
}

int apfc_step_adjoint(apfc_ctx* c, const apfc_state* before, const apfc_state* after, double dt,
                      const double* const* lam_after, double* const* lam_before, double* dL_ddB, void* stream,
                      apfc_stats* stats) {
    auto t0 = std::chrono::steady_clock::now();
    if (int rc = need_ws(c); rc) return rc;
    if (c->solver.picard_iters != 1) return fail(APFC_ERR_INVALID, "apfc_step_adjoint needs picard_iters == 1");
    if (int rc = check_states(c, before, false); rc) return rc;
    if (int rc = check_states(c, after, false); rc) return rc;
    if (!lam_after || !lam_before) return fail(APFC_ERR_INVALID, "lam arrays are NULL");
    hipStream_t st = (hipStream_t)stream;
    if (int rc = refresh_dt(c, dt, st); rc) return rc;
    std::vector<const void*> t[4];
    for (int b = 0; b < c->count; ++b) {
        if (!lam_after[b] || !lam_before[b]) return fail(APFC_ERR_INVALID, "lam pointer is NULL");
        t[0].push_back(before[b].eta);
        t[1].push_back(after[b].eta);
        t[2].push_back(lam_after[b]);
        t[3].push_back(lam_before[b]);
    }
    if (int rc = upload_ptrs(c, t, 4, st); rc) return rc;
    Dev d = c->dev();
    launch_planar_in(d, tab(c, 0), c->BB, st);                  // eta^{m-1}
    launch_nonlinear(d, c->BB, c->BB, c->dnode, c->B, st);      // only d(eta^{m-1}) is used
    launch_adjoint_rhs(d, tab(c, 2), c->B, st);                 // B = [0 ; lam]
    launch_fill_zero(c->X, 2 * c->NT, st);
    int iters = 0;
    if (int rc = fgmres(c, st, &iters); rc) {
        (void)fill_stats(c, st, stats, 0.0);
        return rc;
    }
    launch_adjoint_out(d, c->X, c->BB, tab(c, 1), tab(c, 3), c->tpart, st);
    launch_reduce(d, c->tpart, kE1, 1, false, c->kr.redr, kSlots, nullptr, st);
    HIPCHK(hipMemcpyAsync(c->h_dbl, c->kr.redr, sizeof(double) * kSlots * c->S, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    if (dL_ddB)
        for (int b = 0; b < c->count; ++b) dL_ddB[b] += c->h_dbl[(b * c->J) * kSlots];
    const double ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    return fill_stats(c, st, stats, ms);
}

int apfc_apply(apfc_ctx* c, int which, const apfc_state* lin, const apfc_state* in, apfc_state* out, double dt,
               void* stream) {
    if (int rc = need_ws(c); rc) return rc;
    if (which != APFC_OP_A && which != APFC_OP_PINV) return fail(APFC_ERR_INVALID, "apfc_apply: unknown operator");
    if (int rc = check_states(c, in, true); rc) return rc;
    if (int rc = check_states(c, out, true); rc) return rc;
    if (which == APFC_OP_A)
        if (int rc = check_states(c, lin, false); rc) return rc;
    hipStream_t st = (hipStream_t)stream;
    if (int rc = refresh_dt(c, dt, st); rc) return rc;
    std::vector<const void*> t[4];
    for (int b = 0; b < c->count; ++b) {
        t[0].push_back(in[b].eta);
        t[1].push_back(in[b].zeta);
        t[2].push_back(out[b].eta);
        t[3].push_back(out[b].zeta);
    }
    if (int rc = upload_ptrs(c, t, 4, st); rc) return rc;
    Dev d = c->dev();
    d.probe = nullptr;
    if (which == APFC_OP_A) {
        std::vector<const void*> tl[1];
        for (int b = 0; b < c->count; ++b) tl[0].push_back(lin[b].eta);
        launch_state_in(d, tab(c, 0), tab(c, 1), c->W, st);          // W = input (zeta, eta)
        HIPCHK(hipStreamSynchronize(st));
        if (int rc = upload_ptrs(c, tl, 1, st); rc) return rc;
        launch_planar_in(d, tab(c, 0), c->BB, st);                    // linearisation eta
        launch_nonlinear(d, c->BB, c->BB, c->dnode, c->B, st);
        HIPCHK(hipStreamSynchronize(st));
        if (int rc = upload_ptrs(c, t, 4, st); rc) return rc;
        launch_apply<double>(d, c->W, c->dnode, c->R, nullptr, st);
        launch_state_out(d, c->R, tab(c, 2), tab(c, 3), st);
    } else {
        if (c->mixed) {
            launch_state_in(d, tab(c, 0), tab(c, 1), c->W, st);
            launch_narrow(c->W, basis<float>(c), 2 * c->NT, st);
            precond<float>(c, d, basis<float>(c), (zf*)c->Z, nullptr, st);
            launch_widen((const zf*)c->Z, c->R, 2 * c->NT, st);
        } else {
            launch_state_in(d, tab(c, 0), tab(c, 1), c->V, st);
            precond<double>(c, d, c->V, c->R, nullptr, st);
        }
        launch_state_out(d, c->R, tab(c, 2), tab(c, 3), st);
    }
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(st));
    return APFC_OK;
}

int apfc_rotation(apfc_ctx* c, const apfc_state* states, double* const* omega, double* const* h,
                  const apfc_refine_params* rp, void* stream) {
    if (int rc = need_ws(c); rc) return rc;
    if (int rc = check_states(c, states, false); rc) return rc;
    if (!omega || !rp) return fail(APFC_ERR_INVALID, "omega and params are required");
    if (!(rp->n_per_wavelength > 0.0) || !(rp->h_int > 0.0) || !(rp->h_max >= rp->h_int) || !(rp->tiny >= 0.0))
        return fail(APFC_ERR_INVALID, "refine params: need n > 0, 0 < h_int <= h_max, tiny >= 0");
    hipStream_t st = (hipStream_t)stream;
    std::vector<const void*> t[3];
    for (int b = 0; b < c->count; ++b) {
        if (!omega[b] || (h && !h[b])) return fail(APFC_ERR_INVALID, "omega[b] / h[b] is NULL");
        t[0].push_back(states[b].eta);
        t[1].push_back(omega[b]);
        t[2].push_back(h ? h[b] : nullptr);
    }
    if (int rc = upload_ptrs(c, t, 3, st); rc) return rc;
    Dev d = c->dev();
    d.probe = nullptr;
    RefineArgs ra{};
    ra.kmax = 0.0;
    for (int j = 0; j < c->J; ++j) {
        double n2 = 0.0;
        for (int q = 0; q < 3; ++q) n2 += c->lattice.k[j][q] * c->lattice.k[j][q];
        ra.kmax = std::max(ra.kmax, std::sqrt(n2));
    }
    ra.nwl = rp->n_per_wavelength;
    ra.eps = rp->grad_A_eps;
    ra.Amin = rp->A_min;
    ra.hint = rp->h_int;
    ra.hmax = rp->h_max;
    ra.tiny = rp->tiny;
    launch_state_in(d, tab(c, 0), nullptr, c->X, st);
    launch_rotation(d, c->X + c->NT, tab(c, 1), h ? tab(c, 2) : nullptr, ra, st);
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(st));
    return APFC_OK;
}

int apfc_set_tiles(apfc_ctx* c, int tile_rows, int precond_region) {
    if (int rc = need_ws(c); rc) return rc;
    if (tile_rows != 4 && tile_rows != 8 && tile_rows != 16 && tile_rows != 32)
        return fail(APFC_ERR_INVALID, "tile_rows must be 4, 8, 16 or 32");
    if (precond_region < 0 || precond_region >= kChebShapes) return fail(APFC_ERR_INVALID, "precond_region must be in 0..5");
    c->TY = tile_rows;
    build_tiles(*c, c->TY, c->tiles);
    if (c->solver.inner_kind == APFC_INNER_CHEB && c->dim == 2) {
        c->cheb_shape = precond_region;
        build_ctiles(*c);
    }
    invalidate_graphs(*c);
    return upload_tables(*c);
}

int apfc_get_tiles(const apfc_ctx* c, int* tile_rows, int* precond_region) {
    if (!c) return fail(APFC_ERR_INVALID, "ctx is NULL");
    if (tile_rows) *tile_rows = c->TY;
    if (precond_region) *precond_region = c->cheb_shape;
    return APFC_OK;
}

int apfc_set_graphs(apfc_ctx* c, int enable) {
    if (!c) return fail(APFC_ERR_INVALID, "ctx is NULL");
    c->use_graphs = enable != 0;
    return APFC_OK;
}

int apfc_probe_enable(apfc_ctx* c, const char* name, int every) {
    if (!c) return fail(APFC_ERR_INVALID, "ctx is NULL");
    if (every < 1) return fail(APFC_ERR_INVALID, "probe: every must be >= 1");
    const int kid = name ? kernel_id(name) : KID_NONE;
    if (name && kid == KID_NONE) return fail(APFC_ERR_INVALID, std::string("unknown kernel name: ") + name);
    if (!c->probe.created && kid != KID_NONE) {
        for (auto& e : c->probe.ev) HIPCHK(hipEventCreate(&e));
        HIPCHK(hipMalloc(&c->probe.d_frac, sizeof(double) * Probe::kMax));
        c->probe.created = true;
    }
    c->probe.target = kid;
    c->probe.every = every;
    for (auto& v : c->probe.seen) v = 0;
    c->probe.n = 0;
    return APFC_OK;
}

namespace {
// Sums over the recorded launches of family kid (KID_ALL: every family) in which some system worked.
int probe_sum(apfc_ctx* c, int kid, int* launches, double* total_ms, double* bytes_per_launch, long long* seen) {
    double tot = 0.0, bytes = 0.0;
    const int n = c->probe.n;
    int used = 0;
    std::vector<double> frac(n);
    if (n > 0) HIPCHK(hipMemcpy(frac.data(), c->probe.d_frac, sizeof(double) * n, hipMemcpyDeviceToHost));
    for (int i = 0; i < n; ++i) {
        if (kid != KID_ALL && c->probe.kid[i] != kid) continue;
        HIPCHK(hipEventSynchronize(c->probe.ev[2 * i + 1]));
        if (frac[i] <= 0.0) continue;   // every system masked: an empty launch, not a sample of the kernel
        float ms = 0.f;
        HIPCHK(hipEventElapsedTime(&ms, c->probe.ev[2 * i], c->probe.ev[2 * i + 1]));
        tot += ms;
        bytes += c->probe.bytes[i] * frac[i];
        ++used;
    }
    if (launches) *launches = used;
    if (total_ms) *total_ms = tot;
    if (bytes_per_launch) *bytes_per_launch = used > 0 ? bytes / used : 0.0;
    if (seen) {
        *seen = 0;
        for (int k = 0; k < KID_COUNT; ++k)
            if (kid == KID_ALL || k == kid) *seen += c->probe.seen[k];
    }
    return APFC_OK;
}
}  // namespace

int apfc_probe_read(apfc_ctx* c, int* launches, double* total_ms, double* bytes_per_launch) {
    if (!c) return fail(APFC_ERR_INVALID, "ctx is NULL");
    const int kid = c->probe.target == KID_NONE ? KID_ALL : c->probe.target;
    if (int rc = probe_sum(c, kid, launches, total_ms, bytes_per_launch, nullptr); rc) return rc;
    c->probe.n = 0;
    return APFC_OK;
}

int apfc_probe_read_kernel(apfc_ctx* c, const char* name, int* launches, double* total_ms, double* bytes_per_launch,
                           long long* issued) {
    if (!c || !name) return fail(APFC_ERR_INVALID, "NULL argument");
    const int kid = kernel_id(name);
    if (kid == KID_NONE || kid == KID_ALL) return fail(APFC_ERR_INVALID, std::string("unknown kernel name: ") + name);
    return probe_sum(c, kid, launches, total_ms, bytes_per_launch, issued);
}

int apfc_autotune(apfc_ctx* c, void* stream, int* chosen) {
    if (int rc = need_ws(c); rc) return rc;
    hipStream_t st = (hipStream_t)stream;
    // candidates for the tile height of the stencil kernels (operator apply, residual, PCG/3D
    // Chebyshev sweeps); every candidate is timed on the same unmasked kernel mix, three
    // interleaved rounds, best round kept
    const int cand[3] = {8, 16, 32};
    float best_ms[3] = {1e30f, 1e30f, 1e30f};
    hipEvent_t e0, e1;
    HIPCHK(hipEventCreate(&e0));
    HIPCHK(hipEventCreate(&e1));
    launch_fill_zero(c->V, 2 * c->NT, st);
    launch_fill_zero(c->X, 2 * c->NT, st);
    launch_fill_zero(c->B, 2 * c->NT, st);
    const long long vs = c->vstride();
    for (int round = 0; round < 3; ++round)
        for (int ci = 0; ci < 3; ++ci) {
            const int ty = cand[ci];
            c->TY = ty;
            build_tiles(*c, ty, c->tiles);
            if (int rc = upload_tables(*c); rc) return rc;
            Dev d = c->dev();
            d.probe = nullptr;
            auto body = [&]() {
                if (c->mixed) {
                    precond<float>(c, d, basis<float>(c), (zf*)c->Z, nullptr, st);
                    launch_apply_dot<float>(d, (const zf*)c->Z, c->dnode, (zf*)c->W, basis<float>(c), vs, 2, c->apart,
                                            nullptr, st);
                } else {
                    precond<double>(c, d, c->V, (zd*)c->Z, nullptr, st);
                    launch_apply_dot<double>(d, (const zd*)c->Z, c->dnode, c->W, c->V, vs, 2, c->apart, nullptr,
                                             st);
                }
                launch_reduce(d, c->apart, 0, 5, false, c->kr.red1, c->kr.nv1 + 1, nullptr, st);
                launch_restart_residual(c, d, nullptr, st);
            };
            body();
            HIPCHK(hipEventRecord(e0, st));
            for (int r = 0; r < 3; ++r) body();
            HIPCHK(hipEventRecord(e1, st));
            HIPCHK(hipEventSynchronize(e1));
            float ms = 0.f;
            HIPCHK(hipEventElapsedTime(&ms, e0, e1));
            best_ms[ci] = std::min(best_ms[ci], ms);
        }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    int bi = 0;
    for (int ci = 1; ci < 3; ++ci)
        if (best_ms[ci] < best_ms[bi]) bi = ci;
    c->TY = cand[bi];
    build_tiles(*c, c->TY, c->tiles);
    if (int rc = upload_tables(*c); rc) return rc;
    // region shape of the fused 2D Chebyshev preconditioner
    if (c->solver.inner_kind == APFC_INNER_CHEB && c->dim == 2) {
        float best_sh[kChebShapes];
        for (int sh = 0; sh < kChebShapes; ++sh) best_sh[sh] = 1e30f;
        HIPCHK(hipEventCreate(&e0));
        HIPCHK(hipEventCreate(&e1));
        for (int round = 0; round < 3; ++round)
            for (int sh = 0; sh < kChebShapes; ++sh) {
                c->cheb_shape = sh;
                build_ctiles(*c);
                if (int rc = upload_tables(*c); rc) return rc;
                Dev d = c->dev();
                d.probe = nullptr;
                auto body = [&]() {
                    if (c->mixed)
                        precond<float>(c, d, basis<float>(c), (zf*)c->Z, nullptr, st);
                    else
                        precond<double>(c, d, c->V, (zd*)c->Z, nullptr, st);
                };
                body();
                HIPCHK(hipEventRecord(e0, st));
                for (int r = 0; r < 3; ++r) body();
                HIPCHK(hipEventRecord(e1, st));
                HIPCHK(hipEventSynchronize(e1));
                float ms = 0.f;
                HIPCHK(hipEventElapsedTime(&ms, e0, e1));
                best_sh[sh] = std::min(best_sh[sh], ms);
            }
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        int bs = 0;
        for (int sh = 1; sh < kChebShapes; ++sh)
            if (best_sh[sh] < best_sh[bs]) bs = sh;
        c->cheb_shape = bs;
        build_ctiles(*c);
        if (int rc = upload_tables(*c); rc) return rc;
    }
    invalidate_graphs(*c);
    if (chosen) *chosen = c->TY;
    return APFC_OK;
}

}  // extern "C"

// ----------------------------------------------------------------------------------------------
// apfc_step_noalloc: one step on the library's static device scratch, for callers that cannot
// allocate.  Every GPU that runs it holds its own copy of `scratch` (kNoAllocBytes, until the process
// ends); its address is looked up once per device and only that address is used on the host side.
// The calls on one GPU share the scratch: a context lays out its tables there again whenever another
// context used it in between (and then restarts the history of the extrapolated guess), and calls
// that overlap in time on one GPU race.
// ----------------------------------------------------------------------------------------------
namespace {
constexpr size_t kNoAllocBytes = size_t(64) << 20;
constexpr int kNoAllocDevices = 64;
void* g_scratch_ptr[kNoAllocDevices] = {};
const apfc_ctx* g_scratch_owner[kNoAllocDevices] = {};

__global__ void k_zero_ints(int* p, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0;
}
}  // namespace

static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

void noalloc_forget(const apfc_ctx* c) {
    for (auto& o : g_scratch_owner)
        if (o == c) o = nullptr;
}

namespace {
// The pointer tables of one step (eta, zeta, source) staged without allocating.
int prepare_step_na(apfc_ctx* c, apfc_state* states, double dt, const double* const* source, hipStream_t st) {
    if (int rc = check_states(c, states, true); rc) return rc;
    if (int rc = refresh_dt(c, dt, st); rc) return rc;
    const int n = c->count;
    for (int b = 0; b < n; ++b) {
        if (source && !source[b]) return fail(APFC_ERR_INVALID, "source[b] is NULL");
        c->na_ptrs[b] = states[b].eta;
        c->na_ptrs[n + b] = states[b].zeta;
        c->na_ptrs[2 * n + b] = source ? source[b] : nullptr;
    }
    return upload_ptrs_na(c, 3 * n, st);
}

// Carve the context's buffers from this device's scratch (first use on the device: look its address
// up) and lay out the tables there, unless this context was the last to do so.
int attach_scratch(apfc_ctx* c, hipStream_t st) {
    int dev = 0;
    HIPCHK(hipGetDevice(&dev));
    if (dev < 0 || dev >= kNoAllocDevices) return fail(APFC_ERR_INVALID, "apfc_step_noalloc: device index out of range");
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        HIPCHK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p || ((uintptr_t)p & 255) != 0) return fail(APFC_ERR_HIP, "apfc_step_noalloc: scratch address not 256-byte aligned");
        g_scratch_ptr[dev] = p;
    }
    char* base = (char*)g_scratch_ptr[dev];
    if (c->ws == base && g_scratch_owner[dev] == c) return APFC_OK;
    c->ws = base;
    c->ws_bytes = kNoAllocBytes;
    carve(*c, base);
    c->hist_n = 0;
    c->tab_shadow.clear();
    c->graphs_valid = false;
    g_scratch_owner[dev] = nullptr;
    // tables by synchronous copies from the context's host vectors; the tickets of the fused reductions
    // start at zero (a fill kernel, not a memset)
    HIPCHK(hipStreamSynchronize(st));
    HIPCHK(hipMemcpyAsync(c->d_sys, c->sys.data(), sizeof(Sys) * c->S, hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(c->d_tiles, c->tiles.data(), sizeof(Tile) * c->tiles.size(), hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(c->d_chunks, c->chunks.data(), sizeof(Chunk) * c->chunks.size(), hipMemcpyHostToDevice, st));
    if (!c->ctiles.empty())
        HIPCHK(hipMemcpyAsync(c->d_ctiles, c->ctiles.data(), sizeof(CTile) * c->ctiles.size(), hipMemcpyHostToDevice, st));
    if (!c->mtiles.empty())
        HIPCHK(hipMemcpyAsync(c->d_mtiles, c->mtiles.data(), sizeof(Tile) * c->mtiles.size(), hipMemcpyHostToDevice, st));
    for (int l = 0; l < c->mg_n; ++l) {
        HIPCHK(hipMemcpyAsync(c->d_mg_sys[l], c->mg_sys[l].data(), sizeof(Sys) * c->S, hipMemcpyHostToDevice, st));
        HIPCHK(hipMemcpyAsync(c->d_mg_tiles[l], c->mg_tiles[l].data(), sizeof(Tile) * c->mg_tiles[l].size(),
                              hipMemcpyHostToDevice, st));
    }
    hipLaunchKernelGGL(k_zero_ints, dim3((c->S + 255) / 256), dim3(256), 0, st, c->kr.tick_c, c->S);
    hipLaunchKernelGGL(k_zero_ints, dim3(1), dim3(64), 0, st, c->kr.tick_p, 1);
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(st));
    g_scratch_owner[dev] = c;
    return APFC_OK;
}

struct NoAllocScope {
    apfc_ctx* c;
    explicit NoAllocScope(apfc_ctx* cc) : c(cc) { c->noalloc = true; }
    ~NoAllocScope() { c->noalloc = false; }
};
}  // namespace

extern "C" int apfc_step_noalloc(apfc_ctx* c, apfc_state* states, double dt, const double* const* source, void* stream,
                                 apfc_stats* stats) {
    auto t0 = std::chrono::steady_clock::now();
    if (!c) return fail(APFC_ERR_INVALID, "ctx is NULL");
    if (c->ws_need > kNoAllocBytes)
        return fail(APFC_ERR_WORKSPACE, "apfc_step_noalloc: the context needs " + std::to_string(c->ws_need) +
                                            " bytes of scratch, more than the " + std::to_string(kNoAllocBytes) +
                                            " bytes of the static scratch; use apfc_step with a workspace");
    hipStream_t st = (hipStream_t)stream;
    NoAllocScope scope(c);
    if (int rc = attach_scratch(c, st); rc) return rc;
    if (int rc = prepare_step_na(c, states, dt, source, st); rc) return rc;
    Dev d = c->dev();
    d.probe = nullptr;
    launch_state_in(d, tab(c, 0), tab(c, 1), c->X, st);
    int iters = 0;
    if (int rc = step_body(c, d, dt, source != nullptr, st, &iters); rc) {
        (void)fill_stats(c, st, stats, 0.0);
        return rc;
    }
    launch_state_out(d, c->X, tab(c, 0), tab(c, 1), st);
    HIPCHK(hipGetLastError());
    const double ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    return fill_stats(c, st, stats, ms);
}

extern "C" size_t apfc_noalloc_max_bytes(void) { return kNoAllocBytes; }
