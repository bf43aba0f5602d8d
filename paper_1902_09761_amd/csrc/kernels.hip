// HIP kernels of the APFC time step for gfx950 (CDNA4, wave64): state conversion, right-hand side and
// nodal nonlinearity, Jacobi-PCG and per-iteration Chebyshev preconditioner stages, Krylov chunk kernels,
// Gram-Schmidt reduction, energy, rotation and adjoint pieces, and their launchers.  The operator apply
// lives in kernels_apply.hip, the fused 2D Chebyshev preconditioner in kernels_cheb2d.hip; the shared
// device helpers in kernels_common.h.
#include "kernels_common.h"

namespace apfc {

// ------------------------------------------------------------------------------------------
// state <-> batched vector
// ------------------------------------------------------------------------------------------
template <int DIM, int TY>
__global__ __launch_bounds__(kBlock) void k_state_in(const Sys* sys, const Tile* tiles, const int* mask,
                                                    double* const* eta_tab, double* const* zeta_tab, zd* X,
                                                    long long NT) {
    TILE_PROLOGUE();
    const double* e = eta_tab[s.inst] + (long long)s.j * 2 * s.N;
    const double* z = zeta_tab ? zeta_tab[s.inst] + (long long)s.j * 2 * s.N : nullptr;
    FOR_ROWS(TY) {
        const long long i = ((long long)pz * s.ny + y) * s.nx + x;
        X[NT + s.off + i] = zd{e[i], e[s.N + i]};
        if (z) X[s.off + i] = zd{z[i], z[s.N + i]};
    }
}

template <int DIM, int TY>
__global__ __launch_bounds__(kBlock) void k_state_out(const Sys* sys, const Tile* tiles, const int* mask, const zd* X,
                                                     double* const* eta_tab, double* const* zeta_tab, long long NT) {
    TILE_PROLOGUE();
    double* e = eta_tab[s.inst] + (long long)s.j * 2 * s.N;
    double* z = zeta_tab ? zeta_tab[s.inst] + (long long)s.j * 2 * s.N : nullptr;
    FOR_ROWS(TY) {
        const long long i = ((long long)pz * s.ny + y) * s.nx + x;
        const zd ve = X[NT + s.off + i];
        e[i] = ve.x;
        e[s.N + i] = ve.y;
        if (z) {
            const zd vz = X[s.off + i];
            z[i] = vz.x;
            z[s.N + i] = vz.y;
        }
    }
}

// planar [J][2][N] per instance <-> one batched half vector
template <int DIM, int TY, bool IN>
__global__ __launch_bounds__(kBlock) void k_planar(const Sys* sys, const Tile* tiles, const int* mask,
                                                  double* const* tab, zd* half) {
    TILE_PROLOGUE();
    double* p = tab[s.inst] + (long long)s.j * 2 * s.N;
    FOR_ROWS(TY) {
        const long long i = ((long long)pz * s.ny + y) * s.nx + x;
        if constexpr (IN) {
            half[s.off + i] = zd{p[i], p[s.N + i]};
        } else {
            const zd v = half[s.off + i];
            p[i] = v.x;
            p[s.N + i] = v.y;
        }
    }
}

__global__ __launch_bounds__(kBlock) void k_fill_zero(zd* p, long long n) {
    for (long long i = blockIdx.x * (long long)kBlock + threadIdx.x; i < n; i += (long long)gridDim.x * kBlock)
        p[i] = zd{0.0, 0.0};
}

// ------------------------------------------------------------------------------------------
// bulk energy at one node (Eq. (5) with the resonant terms of the lattice)
// ------------------------------------------------------------------------------------------
__device__ __forceinline__ double term_coef(const Terms& T, int t, const Sys& s) {
    return T.order[t] == 3 ? -2.0 * s.a3 / s.a0 : 8.0 * s.a2 / s.a0;
}
__device__ __forceinline__ zd factor(const Terms& T, int t, int q, const zd* eta) {
    const zd v = eta[T.idx[t][q]];
    return T.cj[t][q] ? cconj(v) : v;
}

// d = dF_j = 2 a1/a0 + 4 (a2/a0) A (same for every j), h_j = F^s_j - d eta_j.
__device__ __forceinline__ void bulk_h(const Terms& T, const Sys& s, const zd* eta, double& d, zd* h) {
    const int J = T.J;
    double A = 0.0;
    for (int l = 0; l < J; ++l) A += abs2(eta[l]);
    A *= 2.0;
    d = 2.0 * s.a1 / s.a0 + 4.0 * s.a2 / s.a0 * A;
    const double c4 = -4.0 * s.a2 / s.a0;
    for (int l = 0; l < J; ++l) h[l] = (c4 * abs2(eta[l])) * eta[l];
    for (int t = 0; t < T.n; ++t) {
        const double c = term_coef(T, t, s);
        const int ord = T.order[t];
        for (int q = 0; q < ord; ++q) {
            zd p{c, 0.0};
            for (int r = 0; r < ord; ++r)
                if (r != q) p = cmul(p, factor(T, t, r, eta));
            const int l = T.idx[t][q];
            h[l] = h[l] + (T.cj[t][q] ? p : cconj(p));
        }
    }
}

// bulk_h with the amplitudes in registers: JM >= T.J compile-time slots (eta zero beyond T.J), the
// amplitude of a resonant factor picked by unrolled selects instead of a run-time array index, so nothing
// goes through scratch memory.  Same operations in the same order as bulk_h.
template <int JM>
__device__ __forceinline__ zd pick(const zd (&e)[JM], int k) {
    zd r = e[0];
#pragma unroll
    for (int q = 1; q < JM; ++q) {
        // k is the same in every lane (a term-table entry); the comparison goes through readfirstlane so
        // that the chain stays a chain of selects instead of an indexed load from a stack copy of e
        const bool sel = __builtin_amdgcn_readfirstlane(k) == q;
        r.x = sel ? e[q].x : r.x;
        r.y = sel ? e[q].y : r.y;
    }
    return r;
}

template <int JM>
__device__ __forceinline__ void bulk_h_reg(const Terms& T, const Sys& s, const zd (&eta)[JM], double& d,
                                           zd (&h)[JM]) {
    double A = 0.0;
#pragma unroll
    for (int l = 0; l < JM; ++l) A += abs2(eta[l]);
    A *= 2.0;
    d = 2.0 * s.a1 / s.a0 + 4.0 * s.a2 / s.a0 * A;
    const double c4 = -4.0 * s.a2 / s.a0;
#pragma unroll
    for (int l = 0; l < JM; ++l) h[l] = (c4 * abs2(eta[l])) * eta[l];
    for (int t = 0; t < T.n; ++t) {
        const double c = term_coef(T, t, s);
        const int ord = T.order[t];
        zd f[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const zd v = pick(eta, q < ord ? T.idx[t][q] : 0);
            f[q] = (q < ord && T.cj[t][q]) ? cconj(v) : v;
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            if (q >= ord) break;
            zd p{c, 0.0};
#pragma unroll
            for (int r = 0; r < 4; ++r)
                if (r < ord && r != q) p = cmul(p, f[r]);
            const zd add = T.cj[t][q] ? p : cconj(p);
            const int l = T.idx[t][q];
#pragma unroll
            for (int m = 0; m < JM; ++m)
                if (m == l) h[m] = h[m] + add;
        }
    }
}

__device__ __forceinline__ double bulk_f(const Terms& T, const Sys& s, const zd* eta) {
    const int J = T.J;
    double A = 0.0, S4 = 0.0;
    for (int l = 0; l < J; ++l) {
        const double a = abs2(eta[l]);
        A += a;
        S4 += a * a;
    }
    A *= 2.0;
    double f = s.a1 / s.a0 * A + s.a2 / s.a0 * (A * A - 2.0 * S4);
    for (int t = 0; t < T.n; ++t) {
        zd p{1.0, 0.0};
        for (int r = 0; r < T.order[t]; ++r) p = cmul(p, factor(T, t, r, eta));
        f += 2.0 * term_coef(T, t, s) * p.x;
    }
    return f;
}

// ------------------------------------------------------------------------------------------
// RHS and nonlinearity (Eq. (10)/(11), nodal quadrature)
// ------------------------------------------------------------------------------------------
// BB_j = M eta_j / dt (+ M s_j)
template <int DIM, int TY>
__global__ __launch_bounds__(kBlock) void k_rhs_base(const Sys* sys, const Tile* tiles, const int* mask,
                                                    const zd* Xeta, double* const* src_tab, zd* BB) {
    TILE_PROLOGUE();
    const double* src = src_tab ? src_tab[s.inst] + (long long)s.j * 2 * s.N : nullptr;
    FOR_ROWS(TY) {
        Nbr<DIM> n;
        make_nbr<DIM>(s, x, y, pz, n);
        zd Mu, Ku, Tu;
        stencil<DIM, false, false, double>(
            [&](int a, int b, int c) { return Xeta[s.off + nb_index<DIM>(n, a, b, c)]; }, s.h, s.kv[0], s.kv[1],
            s.kv[2], Mu, Ku, Tu);
        zd out = s.inv_dt * Mu;
        if (src) {
            zd Ms;
            stencil<DIM, false, false, double>(
                [&](int a, int b, int c) {
                    const long long i = nb_index<DIM>(n, a, b, c);
                    return zd{src[i], src[s.N + i]};
                },
                s.h, 0.0, 0.0, 0.0, Ms, Ku, Tu);
            out = out + Ms;
        }
        BB[s.off + nb_index<DIM>(n, 1, 1, 1)] = out;
    }
}

// 3D k_rhs_base on z-marching bricks: the x/y passes of each plane of eta_j (and s_j) from LDS, the z pass in
// registers (the arithmetic of the plane-marching stencil kernels).
template <int TY, bool SRC>
__global__ __launch_bounds__(kBlock) void k_rhs_base3d(const Sys* sys, const Tile* tiles, const zd* Xeta,
                                                      double* const* src_tab, zd* BB) {
    const int* mask = nullptr;
    TILE_PROLOGUE();
    constexpr int NF = SRC ? 2 : 1;
    const double* src = SRC ? src_tab[s.inst] + (long long)s.j * 2 * s.N : nullptr;
    const int y = tile.y0 + ty;
    const double h = s.h, m0 = h / 6.0, m1 = 4.0 * h / 6.0, ih = 1.0 / h;
    __shared__ zd buf[2][NF][kPP];
    zmarch_lds<TY / 4, NF, false, false, double, double>(
        s, tile, (int)(threadIdx.x & 63), ty, buf, m0, m1, ih,
        [&](int f, long long i) { return f == 0 ? Xeta[s.off + i] : zd{src[i], src[s.N + i]}; },
        [&](int z, const auto& P) {
            if (x >= s.nx || y >= s.ny || z >= s.nz) return;
            zd Mu, Ku, Tu;
            zcombine<false, false, double>(P[0][0], P[0][1], P[0][2], m0, m1, ih, 0.0, 0.0, 0.0, Mu, Ku, Tu);
            zd out = s.inv_dt * Mu;
            if constexpr (SRC) {
                zd Ms;
                zcombine<false, false, double>(P[NF - 1][0], P[NF - 1][1], P[NF - 1][2], m0, m1, ih, 0.0, 0.0, 0.0, Ms,
                                               Ku, Tu);
                out = out + Ms;
            }
            BB[s.off + ((long long)z * s.ny + y) * s.nx + x] = out;
        });
}

// d (per instance node) and B = [0 ; BB - kappa_j w h_j(eta_it)] for every amplitude of the instance.  The
// J tiles of an instance that cover the same nodes share the rows (amplitude j's tile takes the row steps
// rr with rr % J == j), as in k_rhs_nonlinear.
template <int DIM, int TY, int JM>
__global__ __launch_bounds__(kBlock) void k_nonlinear(const Sys* sys, const Tile* tiles, const Terms T,
                                                     const zd* eta_half, const zd* BB, double* dnode, zd* B,
                                                     long long NT) {
    const int* mask = nullptr;
    TILE_PROLOGUE();
    const int s0 = tile.sys - s.j;   // amplitude 0 of the instance
    const Sys b = sys[s0];
    FOR_ROWS(TY) {
        if (rr_ % T.J != s.j) continue;
        const long long i = ((long long)pz * s.ny + y) * s.nx + x;
        zd eta[JM], h[JM];
#pragma unroll
        for (int l = 0; l < JM; ++l) eta[l] = l < T.J ? eta_half[b.off + l * b.N + i] : zd{0.0, 0.0};
        double d;
        bulk_h_reg<JM>(T, b, eta, d, h);
        dnode[s.doff + i] = d;
#pragma unroll
        for (int l = 0; l < JM; ++l) {
            if (l >= T.J) break;
            const double kap = sys[s0 + l].kappa;
            const long long o = b.off + l * b.N + i;
            B[o] = zd{0.0, 0.0};
            B[NT + o] = BB[o] - (kap * b.w) * h[l];
        }
    }
}

// k_rhs_base and k_nonlinear in one pass for a step with one linearisation (K = 1): the nodal
// nonlinearity of the instance is evaluated once per node and M eta_j/dt (+ M s_j) of every amplitude is
// formed there and used at once, instead of going through BB.  The J tiles of an instance that cover the
// same nodes share the rows (amplitude j's tile takes the row steps rr with rr % J == j).  The same
// arithmetic as the two kernels.
template <int DIM, int TY, int JM>
__global__ __launch_bounds__(kBlock) void k_rhs_nonlinear(const Sys* sys, const Tile* tiles, const Terms T,
                                                         const zd* eta_half, double* const* src_tab, double* dnode,
                                                         zd* B, long long NT) {
    const int* mask = nullptr;
    TILE_PROLOGUE();
    const int s0 = tile.sys - s.j;   // amplitude 0 of the instance
    const Sys b = sys[s0];
    const double* src0 = src_tab ? src_tab[s.inst] : nullptr;
    FOR_ROWS(TY) {
        if (rr_ % T.J != s.j) continue;
        Nbr<DIM> n;
        make_nbr<DIM>(s, x, y, pz, n);
        const long long i = nb_index<DIM>(n, 1, 1, 1);
        zd eta[JM], h[JM];
#pragma unroll
        for (int l = 0; l < JM; ++l) eta[l] = l < T.J ? eta_half[b.off + l * b.N + i] : zd{0.0, 0.0};
        double d;
        bulk_h_reg<JM>(T, b, eta, d, h);
        dnode[s.doff + i] = d;
#pragma unroll
        for (int l = 0; l < JM; ++l) {
            if (l >= T.J) break;
            const Sys& sl = sys[s0 + l];
            zd Mu, Ku, Tu;
            stencil<DIM, false, false, double>(
                [&](int a, int bb, int c) { return eta_half[sl.off + nb_index<DIM>(n, a, bb, c)]; }, sl.h, sl.kv[0],
                sl.kv[1], sl.kv[2], Mu, Ku, Tu);
            zd rhs = sl.inv_dt * Mu;
            if (src0) {
                const double* src = src0 + (long long)l * 2 * s.N;
                zd Ms;
                stencil<DIM, false, false, double>(
                    [&](int a, int bb, int c) {
                        const long long q = nb_index<DIM>(n, a, bb, c);
                        return zd{src[q], src[s.N + q]};
                    },
                    sl.h, 0.0, 0.0, 0.0, Ms, Ku, Tu);
                rhs = rhs + Ms;
            }
            const long long o = sl.off + i;
            B[o] = zd{0.0, 0.0};
            B[NT + o] = rhs - (sl.kappa * s.w) * h[l];
        }
    }
}

// ------------------------------------------------------------------------------------------
// Block preconditioner (Eq. (12), four steps) with fixed-count Jacobi-PCG inner solves.
// Operator of an inner solve: OP = 0 -> M (diag diagM), OP = 1 -> L = M/sqrt(dt) + sqrt(kappa) K.
// The Jacobi diagonal is a constant on the uniform periodic mesh.
// Partials: rho ping-pong slots kRho0/kRho1 = sum |r|^2 / D, slot kPQ = Re p^H q.
// ------------------------------------------------------------------------------------------
template <int OP>
__device__ __forceinline__ double op_diag(const Sys& s) { return OP == 0 ? s.diagM : s.diagL; }

// step 1 init: r = beta1 (zeta part of v), p0 = r / D_M
template <int DIM, int TY, typename T>
__global__ __launch_bounds__(kBlock) void k_cg_init_copy(const Sys* sys, const Tile* tiles, const int* mask,
                                                        const cx<T>* v, cx<T>* r, cx<T>* p0, double* part,
                                                        int ntiles) {
    __shared__ double lds[4];
    TILE_PROLOGUE();
    const double iD = 1.0 / s.diagM;
    double acc[1] = {0.0};
    FOR_ROWS(TY) {
        const long long i = s.off + ((long long)pz * s.ny + y) * s.nx + x;
        const cx<T> rv = ld<T>(v, i);
        r[i] = rv;
        p0[i] = T(iD) * rv;
        acc[0] += (double(rv.x) * double(rv.x) + double(rv.y) * double(rv.y)) * iD;
    }
    block_sum<1>(acc, lds);
    if (threadIdx.x == 0) part[kRho0 * (long long)ntiles + blockIdx.x] = acc[0];
}

// step 2 init: r = beta2 - kappa G x1 (x1 ~ M^{-1} beta1), p0 = r / D_L
template <int DIM, int TY, typename T>
__global__ __launch_bounds__(kBlock) void k_cg_init_g(const Sys* sys, const Tile* tiles, const int* mask,
                                                     const cx<T>* v, const cx<T>* x1, cx<T>* r, cx<T>* p0,
                                                     double* part, int ntiles, long long NT) {
    __shared__ double lds[4];
    TILE_PROLOGUE();
    const T iD = T(1.0 / s.diagL);
    double acc[1] = {0.0};
    FOR_ROWS(TY) {
        Nbr<DIM> n;
        make_nbr<DIM>(s, x, y, pz, n);
        cx<T> Mu, Ku, Tu;
        stencil<DIM, true, true, T>([&](int a, int b, int c) { return ld<T>(x1, s.off + nb_index<DIM>(n, a, b, c)); },
                                    T(s.h), T(s.kv[0]), T(s.kv[1]), T(s.kv[2]), Mu, Ku, Tu);
        const long long i = s.off + nb_index<DIM>(n, 1, 1, 1);
        const cx<T> rv = ld<T>(v, NT + i) - T(s.kappa) * gop(Ku, Tu);
        r[i] = rv;
        p0[i] = iD * rv;
        acc[0] += (double(rv.x) * double(rv.x) + double(rv.y) * double(rv.y)) / s.diagL;
    }
    block_sum<1>(acc, lds);
    if (threadIdx.x == 0) part[kRho0 * (long long)ntiles + blockIdx.x] = acc[0];
}

// step 3 init: r = M x2 (x2 ~ beta2'), p0 = r / D_L.  Also the energy's mass solve uses
// GETA = true: r = G_j eta_j (rhs of M zeta = G eta), p0 = r / D_M.
template <int DIM, int TY, typename T, bool GETA>
__global__ __launch_bounds__(kBlock) void k_cg_init_m(const Sys* sys, const Tile* tiles, const int* mask,
                                                     const cx<T>* x2, cx<T>* r, cx<T>* p0, double* part,
                                                     int ntiles) {
    __shared__ double lds[4];
    TILE_PROLOGUE();
    const double D = GETA ? s.diagM : s.diagL;
    const T iD = T(1.0 / D);
    double acc[1] = {0.0};
    FOR_ROWS(TY) {
        Nbr<DIM> n;
        make_nbr<DIM>(s, x, y, pz, n);
        cx<T> Mu, Ku, Tu;
        stencil<DIM, GETA, GETA, T>([&](int a, int b, int c) { return ld<T>(x2, s.off + nb_index<DIM>(n, a, b, c)); },
                                    T(s.h), T(s.kv[0]), T(s.kv[1]), T(s.kv[2]), Mu, Ku, Tu);
        const long long i = s.off + nb_index<DIM>(n, 1, 1, 1);
        const cx<T> rv = GETA ? gop(Ku, Tu) : Mu;
        r[i] = rv;
        p0[i] = iD * rv;
        acc[0] += (double(rv.x) * double(rv.x) + double(rv.y) * double(rv.y)) / D;
    }
    block_sum<1>(acc, lds);
    if (threadIdx.x == 0) part[kRho0 * (long long)ntiles + blockIdx.x] = acc[0];
}

// q = OP p with p = r/D + beta p_prev (FIRST: p = pin as is); partial Re p^H q.
template <int DIM, int TY, typename T, int OP, bool FIRST>
__global__ __launch_bounds__(kBlock) void k_cg_spmv(const Sys* sys, const Tile* tiles, const int* mask,
                                                   const cx<T>* r, const cx<T>* pin, cx<T>* pout, cx<T>* q,
                                                   double* part, int ntiles, int it) {
    __shared__ double lds[8];
    TILE_PROLOGUE();
    const double D = op_diag<OP>(s);
    T beta = T(0);
    if constexpr (!FIRST) {
        const int sl[2] = {it & 1, (it - 1) & 1};
        double rho[2];
        sum_partials<2>(part, ntiles, sl, s.tbeg, s.tend, rho, lds);
        beta = rho[1] != 0.0 ? T(rho[0] / rho[1]) : T(0);
    }
    const T iD = T(1.0 / D);
    const T cM = OP == 0 ? T(1) : T(s.isq_dt), cK = OP == 0 ? T(0) : T(s.sq_kap);
    double acc[1] = {0.0};
    FOR_ROWS(TY) {
        Nbr<DIM> n;
        make_nbr<DIM>(s, x, y, pz, n);
        auto fp = [&](int a, int b, int c) {
            const long long i = s.off + nb_index<DIM>(n, a, b, c);
            if constexpr (FIRST)
                return ld<T>(pin, i);
            else
                return iD * ld<T>(r, i) + beta * ld<T>(pin, i);
        };
        cx<T> Mu, Ku, Tu;
        stencil<DIM, OP == 1, false, T>(fp, T(s.h), T(0), T(0), T(0), Mu, Ku, Tu);
        const cx<T> qv = OP == 0 ? Mu : cM * Mu + cK * Ku;
        const long long i = s.off + nb_index<DIM>(n, 1, 1, 1);
        const cx<T> pc = fp(1, 1, 1);
        if constexpr (!FIRST) pout[i] = pc;
        q[i] = qv;
        acc[0] += double(pc.x) * double(qv.x) + double(pc.y) * double(qv.y);
    }
    block_sum<1>(acc, lds);
    if (threadIdx.x == 0) part[kPQ * (long long)ntiles + blockIdx.x] = acc[0];
}

// alpha = rho / p^H q; x = x + alpha p (FIRST: x = alpha p); r -= alpha q and partial of the
// next rho unless LAST.
template <int DIM, int TY, typename T, int OP, bool FIRST, bool LAST>
__global__ __launch_bounds__(kBlock) void k_cg_update(const Sys* sys, const Tile* tiles, const int* mask,
                                                     cx<T>* xv, cx<T>* r, const cx<T>* p, const cx<T>* q,
                                                     double* part, int ntiles, int it) {
    __shared__ double lds[8];
    TILE_PROLOGUE();
    const int sl[2] = {it & 1, kPQ};
    double red[2];
    sum_partials<2>(part, ntiles, sl, s.tbeg, s.tend, red, lds);
    const T alpha = (red[0] != 0.0 && red[1] != 0.0) ? T(red[0] / red[1]) : T(0);
    const double D = op_diag<OP>(s);
    double acc[1] = {0.0};
    FOR_ROWS(TY) {
        const long long i = s.off + ((long long)pz * s.ny + y) * s.nx + x;
        const cx<T> pv = ld<T>(p, i);
        if constexpr (FIRST)
            xv[i] = alpha * pv;
        else
            xv[i] = ld<T>(xv, i) + alpha * pv;
        if constexpr (!LAST) {
            const cx<T> rv = ld<T>(r, i) - alpha * ld<T>(q, i);
            r[i] = rv;
            acc[0] += (double(rv.x) * double(rv.x) + double(rv.y) * double(rv.y)) / D;
        }
    }
    if constexpr (!LAST) {
        block_sum<1>(acc, lds);
        if (threadIdx.x == 0) part[((it + 1) & 1) * (long long)ntiles + blockIdx.x] = acc[0];
    }
}

// step 4: chi1 = beta1' - (beta2' - chi2 / sqrt(dt)) / sqrt(kappa); chi2 already in z's eta part
template <int DIM, int TY, typename T>
__global__ __launch_bounds__(kBlock) void k_pc_final(const Sys* sys, const Tile* tiles, const int* mask,
                                                    const cx<T>* x1, const cx<T>* x2, cx<T>* z, long long NT) {
    TILE_PROLOGUE();
    const T isd = T(s.isq_dt), isk = T(s.isq_kap);
    FOR_ROWS(TY) {
        const long long i = s.off + ((long long)pz * s.ny + y) * s.nx + x;
        z[i] = ld<T>(x1, i) - isk * (ld<T>(x2, i) - isd * ld<T>(z, NT + i));
    }
}

// ------------------------------------------------------------------------------------------
// Block preconditioner with Chebyshev-Jacobi inner solves, one launch per inner iteration (any
// dimension; used in 3D, where a halo of several layers of a 27-point stencil does not fit LDS).
// Same recurrence as k_cheb2d, with the scalars of iteration j from the system's table (Sys::cb).
// ------------------------------------------------------------------------------------------

// r0 of the inner solve (STAGE 0: beta1; 1: beta2 - kappa G x1; 2: M x2; 3: G src for the accurate
// mass solve M zeta = G eta), d0 = r0/(theta D), x = d0
template <int DIM, int TY, typename T, int STAGE>
__global__ __launch_bounds__(kBlock) void k_cb_init(const Sys* sys, const Tile* tiles, const int* mask, const cx<T>* v,
                                                   const cx<T>* src, cx<T>* r, cx<T>* d, cx<T>* xv, long long NT) {
    TILE_PROLOGUE();
    constexpr bool isM = STAGE == 0 || STAGE == 3;
    constexpr bool WG = STAGE == 1 || STAGE == 3;
    const T scale = T(sys[tile.sys].cb[isM ? 0 : 1][0][0]);
    FOR_ROWS(TY) {
        Nbr<DIM> n;
        make_nbr<DIM>(s, x, y, pz, n);
        const long long i = s.off + nb_index<DIM>(n, 1, 1, 1);
        cx<T> rv;
        if constexpr (STAGE == 0) {
            rv = ld<T>(v, i);
        } else {
            cx<T> Mu, Ku, Tu;
            stencil<DIM, WG, WG, T>(
                [&](int a, int b, int c) { return ld<T>(src, s.off + nb_index<DIM>(n, a, b, c)); }, T(s.h),
                T(s.kv[0]), T(s.kv[1]), T(s.kv[2]), Mu, Ku, Tu);
            if constexpr (STAGE == 1)
                rv = ld<T>(v, NT + i) - T(s.kappa) * gop(Ku, Tu);
            else if constexpr (STAGE == 3)
                rv = gop(Ku, Tu);
            else
                rv = Mu;
        }
        const cx<T> dv = scale * rv;
        r[i] = rv;
        d[i] = dv;
        xv[i] = dv;
    }
}

// iteration j >= 1: q = OP d_{j-1}; r -= q; d_j = c1 d_{j-1} + c2 D^{-1} r; x += d_j
template <int DIM, int TY, typename T, int OP, bool LAST>
__global__ __launch_bounds__(kBlock) void k_cb_iter(const Sys* sys, const Tile* tiles, const int* mask, int j,
                                                   const cx<T>* din, cx<T>* dout, cx<T>* r, cx<T>* xv) {
    TILE_PROLOGUE();
    const T c1 = T(sys[tile.sys].cb[OP][j][0]), c2 = T(sys[tile.sys].cb[OP][j][1]);
    const T cM = OP == 0 ? T(1) : T(s.isq_dt), cK = OP == 0 ? T(0) : T(s.sq_kap);
    FOR_ROWS(TY) {
        Nbr<DIM> n;
        make_nbr<DIM>(s, x, y, pz, n);
        cx<T> Mu, Ku, Tu;
        stencil<DIM, OP == 1, false, T>([&](int a, int b, int c) { return ld<T>(din, s.off + nb_index<DIM>(n, a, b, c)); },
                                        T(s.h), T(0), T(0), T(0), Mu, Ku, Tu);
        const long long i = s.off + nb_index<DIM>(n, 1, 1, 1);
        const cx<T> q = OP == 0 ? Mu : cM * Mu + cK * Ku;
        const cx<T> rv = ld<T>(r, i) - q;
        const cx<T> dv = c1 * ld<T>(din, i) + c2 * rv;
        xv[i] = ld<T>(xv, i) + dv;
        if constexpr (!LAST) {
            r[i] = rv;
            dout[i] = dv;
        }
    }
}

// 3D versions of k_cb_init (STAGE 1..3, the stages with a stencil) and k_cb_iter on z-marching
// bricks; same arithmetic per node.
// RR planes per thread on bricks of 64 x BY columns (64 x BY threads).
template <int RR, int BY, typename T, int STAGE>
__global__ __launch_bounds__(64 * BY) void k_cb_init3d(const Sys* sys, const Tile* tiles, const int* mask,
                                                      const cx<T>* v, const cx<T>* src, cx<T>* r, cx<T>* d, cx<T>* xv,
                                                      long long NT) {
    static_assert(STAGE >= 1 && STAGE <= 3, "stage 0 has no stencil");
    TILE_PROLOGUE();
    constexpr bool isM = STAGE == 3;
    constexpr bool WG = STAGE == 1 || STAGE == 3;
    const T scale = T(sys[tile.sys].cb[isM ? 0 : 1][0][0]);
    const int y = tile.y0 + ty;
    const T h = T(s.h), m0 = h * T(1.0 / 6.0), m1 = h * T(4.0 / 6.0), ih = T(1) / h;
    const T k0 = T(s.kv[0]), k1 = T(s.kv[1]), k2 = T(s.kv[2]);
    __shared__ cx<T> buf[2][1][kPPb<BY>];
    zmarch_lds<RR, 1, WG, WG, T, T, BY>(
        s, tile, (int)(threadIdx.x & 63), ty, buf, m0, m1, ih, [&](int, long long i) { return src[s.off + i]; },
        [&](int z, const auto& P) {
            if (x >= s.nx || y >= s.ny || z >= s.nz) return;
            const long long i = s.off + ((long long)z * s.ny + y) * s.nx + x;
            cx<T> Mu, Ku, Tu;
            zcombine<WG, WG, T>(P[0][0], P[0][1], P[0][2], m0, m1, ih, k0, k1, k2, Mu, Ku, Tu);
            cx<T> rv;
            if constexpr (STAGE == 1)
                rv = ld<T>(v, NT + i) - T(s.kappa) * gop(Ku, Tu);
            else if constexpr (STAGE == 3)
                rv = gop(Ku, Tu);
            else
                rv = Mu;
            const cx<T> dv = scale * rv;
            r[i] = rv;
            if (d) d[i] = dv;   // not kept by the three-term form (k_cx_iter3d)
            if (xv) xv[i] = dv;   // the three-term form re-forms x_1 = d_0 from r where it needs it
        });
}

// FINAL (the last iteration of step 3): also step 4 of the preconditioner, z_zeta = x1 - (x2 - chi2 /
// sqrt(dt)) / sqrt(kappa) with chi2 the new iterate (xv = the eta part of z, zz = its zeta part).
template <int TY, typename T, int OP, bool LAST, bool FINAL = false>
__global__ __launch_bounds__(kBlock) void k_cb_iter3d(const Sys* sys, const Tile* tiles, const int* mask, int j,
                                                     const cx<T>* din, cx<T>* dout, cx<T>* r, cx<T>* xv,
                                                     const cx<T>* x1 = nullptr, const cx<T>* x2 = nullptr,
                                                     cx<T>* zz = nullptr) {
    TILE_PROLOGUE();
    const T c1 = T(sys[tile.sys].cb[OP][j][0]), c2 = T(sys[tile.sys].cb[OP][j][1]);
    const T cM = OP == 0 ? T(1) : T(s.isq_dt), cK = OP == 0 ? T(0) : T(s.sq_kap);
    const int y = tile.y0 + ty;
    const T h = T(s.h), m0 = h * T(1.0 / 6.0), m1 = h * T(4.0 / 6.0), ih = T(1) / h;
    __shared__ cx<T> buf[2][1][kPP];
    zmarch_lds<TY / 4, 1, OP == 1, false, T, T>(
        s, tile, (int)(threadIdx.x & 63), ty, buf, m0, m1, ih, [&](int, long long i) { return din[s.off + i]; },
        [&](int z, const auto& P) {
            if (x >= s.nx || y >= s.ny || z >= s.nz) return;
            const long long i = s.off + ((long long)z * s.ny + y) * s.nx + x;
            cx<T> Mu, Ku, Tu;
            zcombine<OP == 1, false, T>(P[0][0], P[0][1], P[0][2], m0, m1, ih, T(0), T(0), T(0), Mu, Ku, Tu);
            const cx<T> q = OP == 0 ? Mu : cM * Mu + cK * Ku;
            const cx<T> rv = ld<T>(r, i) - q;
            const cx<T> dv = c1 * P[0][1].c + c2 * rv;
            const cx<T> xn = ld<T>(xv, i) + dv;
            xv[i] = xn;
            if constexpr (!LAST) {
                r[i] = rv;
                dout[i] = dv;
            }
            if constexpr (FINAL) zz[i] = ld<T>(x1, i) - T(s.isq_kap) * (ld<T>(x2, i) - T(s.isq_dt) * xn);
        });
}

// Step 1's initialisation and first Chebyshev iteration in one plane march (3D): r0 = beta1 (the zeta part
// of v), d0 = x0 = r0/(theta D) formed from v as the planes are staged, then r1 = r0 - M d0,
// d1 = c1 d0 + c2 D^{-1} r1, x1 = x0 + d1.  Same arithmetic as k_cb_init (stage 0) + k_cb_iter3d (j = 1).
template <int TY, typename T, bool LAST>
__global__ __launch_bounds__(kBlock) void k_cb_first3d(const Sys* sys, const Tile* tiles, const int* mask,
                                                      const cx<T>* v, cx<T>* dout, cx<T>* r, cx<T>* xv) {
    TILE_PROLOGUE();
    const T scale = T(sys[tile.sys].cb[0][0][0]);
    const T c1 = T(sys[tile.sys].cb[0][1][0]), c2 = T(sys[tile.sys].cb[0][1][1]);
    const int y = tile.y0 + ty;
    const T h = T(s.h), m0 = h * T(1.0 / 6.0), m1 = h * T(4.0 / 6.0), ih = T(1) / h;
    __shared__ cx<T> buf[2][1][kPP];
    zmarch_lds<TY / 4, 1, false, false, T, T>(
        s, tile, (int)(threadIdx.x & 63), ty, buf, m0, m1, ih,
        [&](int, long long i) { return scale * ld<T>(v, s.off + i); },
        [&](int z, const auto& P) {
            if (x >= s.nx || y >= s.ny || z >= s.nz) return;
            const long long i = s.off + ((long long)z * s.ny + y) * s.nx + x;
            cx<T> Mu, Ku, Tu;
            zcombine<false, false, T>(P[0][0], P[0][1], P[0][2], m0, m1, ih, T(0), T(0), T(0), Mu, Ku, Tu);
            const cx<T> d0 = P[0][1].c;
            const cx<T> rv = ld<T>(v, i) - Mu;
            const cx<T> dv = c1 * d0 + c2 * rv;
            xv[i] = d0 + dv;
            if constexpr (!LAST) {
                r[i] = rv;
                dout[i] = dv;
            }
        });
}

// Iteration j >= 1 of the Chebyshev solve for L in three-term form on the iterates (3D):
//   x_{j+1} = x_j + c1 (x_j - x_{j-1}) + c2 (b - L x_j),   x_0 = 0,
// with the scalars (c1, c2) of iteration j of the correction form (k_cb_iter3d: d_j = c1 d_{j-1} + c2 r_j,
// x_{j+1} = x_j + d_j, where d_{j-1} = x_j - x_{j-1} and r_j = b - L x_j), so the iterates are the same in
// exact arithmetic; per node it reads x_j (stencil), x_{j-1} and b and writes x_{j+1}, two vectors fewer
// than the correction form.  x_1 = d_0 = s b (s = the first scalar of the table) is not stored: FIRST
// (j = 1) stages s b in place of x_1, PREVB (j = 2) forms x_{j-1} = s b from the b it reads anyway.  xout
// may be xkm1 (each node is read, then written, by one thread).  FINAL: also step 4,
// z_zeta = x1 - (x2 - chi2 / sqrt(dt)) / sqrt(kappa) with chi2 = x_{j+1}.
template <int RR, int BY, typename T, bool FIRST, bool PREVB, bool FINAL>
__global__ __launch_bounds__(64 * BY) void k_cx_iter3d(const Sys* sys, const Tile* tiles, const int* mask, int j,
                                                      const cx<T>* xk, const cx<T>* xkm1, const cx<T>* b,
                                                      cx<T>* xout, const cx<T>* x1, const cx<T>* x2, cx<T>* zz) {
    TILE_PROLOGUE();
    static_assert(!(FIRST && PREVB), "x_{j-1} is formed from b only at j = 2");
    const T c1 = T(sys[tile.sys].cb[1][j][0]), c2 = T(sys[tile.sys].cb[1][j][1]);
    const T s0 = T(sys[tile.sys].cb[1][0][0]);
    const T cM = T(s.isq_dt), cK = T(s.sq_kap);
    const int y = tile.y0 + ty;
    const T h = T(s.h), m0 = h * T(1.0 / 6.0), m1 = h * T(4.0 / 6.0), ih = T(1) / h;
    __shared__ cx<T> buf[2][1][kPPb<BY>];
    zmarch_lds<RR, 1, true, false, T, T, BY>(
        s, tile, (int)(threadIdx.x & 63), ty, buf, m0, m1, ih,
        [&](int, long long i) {
            if constexpr (FIRST)
                return s0 * b[s.off + i];
            else
                return xk[s.off + i];
        },
        [&](int z, const auto& P) {
            if (x >= s.nx || y >= s.ny || z >= s.nz) return;
            const long long i = s.off + ((long long)z * s.ny + y) * s.nx + x;
            cx<T> Mu, Ku, Tu;
            zcombine<true, false, T>(P[0][0], P[0][1], P[0][2], m0, m1, ih, T(0), T(0), T(0), Mu, Ku, Tu);
            const cx<T> xc = P[0][1].c, bv = ld<T>(b, i);
            const cx<T> dprev = FIRST ? xc : xc - (PREVB ? s0 * bv : ld<T>(xkm1, i));
            const cx<T> xn = xc + c1 * dprev + c2 * (bv - (cM * Mu + cK * Ku));
            xout[i] = xn;
            if constexpr (FINAL) zz[i] = ld<T>(x1, i) - T(s.isq_kap) * (ld<T>(x2, i) - T(s.isq_dt) * xn);
        });
}

// ------------------------------------------------------------------------------------------
// Krylov kernels over chunks of full vectors (element e < N: zeta part, else eta part)
// ------------------------------------------------------------------------------------------
__device__ __forceinline__ long long elem_index(const Sys& s, long long NT, long long e) {
    return e < s.N ? s.off + e : NT + s.off + (e - s.N);
}

#define CHUNK_PROLOGUE()                                 \
    const Chunk ch = chunks[blockIdx.x];                 \
    if (mask && !mask[ch.sys]) return;                   \
    const Sys s = sys[ch.sys];                           \
    const long long twoN = 2 * s.N;

#define FOR_ELEMS()                                                                   \
    _Pragma("unroll") for (int u_ = 0; u_ < kChunk / kBlock; ++u_)                    \
        if (const long long e = (long long)ch.e0 + threadIdx.x + (long long)u_ * kBlock; e < twoN)

// out = (w - sum_l hcoef_l V_l) * hinv, formed in FP64 and stored in the basis precision
template <typename VT>
__global__ __launch_bounds__(kBlock) void k_proj_final(const Sys* sys, const Chunk* chunks, const int* mask,
                                                      const VT* V, long long vstride, int nv, const VT* w,
                                                      const double* hcoef, int hld, const double* hinv, VT* out,
                                                      long long NT) {
    __shared__ zd cf[kMaxRestart + 1];
    CHUNK_PROLOGUE();
    for (int l = threadIdx.x; l < nv; l += kBlock)
        cf[l] = zd{hcoef[ch.sys * hld + 2 * l], hcoef[ch.sys * hld + 2 * l + 1]};
    __syncthreads();
    const double sc = hinv[ch.sys];
    constexpr int EPT = kChunk / kBlock;
    if (ch.e0 + kChunk <= twoN) {
        // full chunk: basis vector by basis vector over the thread's EPT elements, so EPT loads are in
        // flight at a time instead of one
        long long gi[EPT];
        zd wv[EPT];
#pragma unroll
        for (int u = 0; u < EPT; ++u) {
            gi[u] = elem_index(s, NT, (long long)ch.e0 + threadIdx.x + (long long)u * kBlock);
            wv[u] = ld<double>(w, gi[u]);
        }
        for (int l = 0; l < nv; ++l) {
            const zd c = cf[l];
#pragma unroll
            for (int u = 0; u < EPT; ++u) wv[u] = wv[u] - cmul(c, ld<double>(V, l * vstride + gi[u]));
        }
#pragma unroll
        for (int u = 0; u < EPT; ++u) stv(out, gi[u], sc * wv[u]);
        return;
    }
    FOR_ELEMS() {
        const long long gi = elem_index(s, NT, e);
        zd wv = ld<double>(w, gi);
        for (int l = 0; l < nv; ++l) wv = wv - cmul(cf[l], ld<double>(V, l * vstride + gi));
        stv(out, gi, sc * wv);
    }
}

template <typename VT>
__global__ __launch_bounds__(kBlock) void k_scale(const Sys* sys, const Chunk* chunks, const int* mask, const VT* r,
                                                 const double* inv_beta, VT* v0, long long NT) {
    CHUNK_PROLOGUE();
    const double sc = inv_beta[ch.sys];
    FOR_ELEMS() {
        const long long gi = elem_index(s, NT, e);
        stv(v0, gi, sc * ld<double>(r, gi));
    }
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_xupdate(const Sys* sys, const Chunk* chunks, const int* mask,
                                                   const cx<T>* Z, long long zstride, const int* kcount,
                                                   const double* y, int ldy, zd* X, long long NT) {
    __shared__ zd cf[kMaxRestart];
    CHUNK_PROLOGUE();
    const int kc = kcount[ch.sys];
    if (kc <= 0) return;
    for (int l = threadIdx.x; l < kc; l += kBlock) cf[l] = zd{y[ch.sys * ldy + 2 * l], y[ch.sys * ldy + 2 * l + 1]};
    __syncthreads();
    constexpr int EPT = kChunk / kBlock;
    if (ch.e0 + kChunk <= twoN) {
        // full chunk: EPT loads in flight per basis vector (as in k_proj_final)
        long long gi[EPT];
        zd xv[EPT];
#pragma unroll
        for (int u = 0; u < EPT; ++u) {
            gi[u] = elem_index(s, NT, (long long)ch.e0 + threadIdx.x + (long long)u * kBlock);
            xv[u] = X[gi[u]];
        }
        for (int l = 0; l < kc; ++l) {
            const zd c = cf[l];
#pragma unroll
            for (int u = 0; u < EPT; ++u) xv[u] = xv[u] + cmul(c, ld<double>(Z, l * zstride + gi[u]));
        }
#pragma unroll
        for (int u = 0; u < EPT; ++u) X[gi[u]] = xv[u];
        return;
    }
    FOR_ELEMS() {
        const long long gi = elem_index(s, NT, e);
        zd xv = X[gi];
        for (int l = 0; l < kc; ++l) xv = xv + cmul(cf[l], ld<double>(Z, l * zstride + gi));
        X[gi] = xv;
    }
}

// out[s*nvals + v] = sum of part[v*P + t] over the system's tiles or chunks (fixed order)
__global__ __launch_bounds__(kBlock) void k_reduce(const Sys* sys, const int* mask, const double* part, long long P,
                                                  int slot0, int nvals, bool chunk_ranges, double* out, int ld) {
    const int si = blockIdx.x;
    if (mask && !mask[si]) return;
    const Sys s = sys[si];
    const int beg = chunk_ranges ? s.cbeg : s.tbeg, end = chunk_ranges ? s.cend : s.tend;
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
    for (int v = blockIdx.y * 4 + wv; v < nvals; v += gridDim.y * 4) {
        double a = 0.0;
        for (int t = beg + lane; t < end; t += 64) a += part[(slot0 + v) * P + t];
        a = wave_sum(a);
        if (lane == 0) out[si * (long long)ld + v] = a;
    }
}

// ------------------------------------------------------------------------------------------
// small per-system FGMRES bookkeeping (one thread per system)
// ------------------------------------------------------------------------------------------
__device__ void cycle_init_sys(const Krylov& kr, int s, int first, double rr, double bb) {
    const double beta = sqrt(rr);
    if (!isfinite(beta) || !isfinite(bb)) {
        kr.err[0] = 1;
        kr.solve_active[s] = 0;
        kr.iter_active[s] = 0;
        return;
    }
    if (first) {
        const double bn = sqrt(bb);
        kr.bnorm[s] = bn;
        // a zero right-hand side is solved relative to the initial residual
        kr.target[s] = kr.rtol * (bn > 0.0 ? bn : beta);
    }
    const double bnorm = kr.bnorm[s];
    kr.relres[s] = bnorm > 0.0 ? beta / bnorm : beta;
    kr.kcount[s] = 0;
    if (beta <= kr.target[s]) {
        kr.solve_active[s] = 0;
        kr.iter_active[s] = 0;
        return;
    }
    kr.solve_active[s] = 1;
    kr.iter_active[s] = 1;
    kr.cycles[s] += 1;
    kr.inv_beta[s] = 1.0 / beta;
    double* g = kr.g + (long long)s * 2 * (kr.m + 1);
    g[0] = beta;
    g[1] = 0.0;
    for (int i = 1; i <= kr.m; ++i) g[2 * i] = g[2 * i + 1] = 0.0;
}

// One workgroup per system: |r|^2 and |b|^2 from the residual partials (slots kRR, kBB, one wave
// each, fixed order), then the cycle's start (beta, target on the first cycle, the state); systems that
// stopped solving are skipped after the first cycle.  With pub, every workgroup takes a ticket and the
// last one writes the host summary.
__global__ __launch_bounds__(kBlock) void k_cycle_start(const Sys* sys, Krylov kr, int S, int first,
                                                        const double* part, long long P, int* pub) {
    __shared__ double red[2];
    __shared__ int flag;
    const int si = blockIdx.x;
    if (first || kr.solve_active[si]) {
        const Sys s = sys[si];
        const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
        if (wv < 2) {
            double a = 0.0;
            for (int t = s.tbeg + lane; t < s.tend; t += 64) a += part[(kRR + wv) * P + t];
            a = wave_sum(a);
            if (lane == 0) {
                red[wv] = a;
                kr.redr[2 * si + wv] = a;
            }
        }
        __syncthreads();
        if (threadIdx.x == 0) cycle_init_sys(kr, si, first, red[0], red[1]);
    }
    if (!pub) return;
    __syncthreads();
    if (threadIdx.x == 0) {
        __threadfence();                      // this workgroup's state before its ticket
        const int t = atomicAdd(kr.tick_p, 1);
        flag = t == S - 1;
        if (flag) *kr.tick_p = 0;
    }
    __syncthreads();
    if (!flag) return;
    __threadfence();                          // the other workgroups' state after their tickets
    if (threadIdx.x == 0) {
        int any = 0, mx = 0;
        for (int q = 0; q < S; ++q) {
            any |= kr.solve_active[q];
            mx = kr.iters[q] > mx ? kr.iters[q] : mx;
        }
        pub[0] = any;
        pub[1] = kr.err[0];
        pub[2] = mx;
    }
}

// Column k of the Hessenberg matrix from the two projections, Givens rotations, residual estimate,
// convergence / breakdown / restart decision for system s.  Reads only LDS (h1, h2; rot = the previous
// rotations cs[0..k), sn[0..2k) and g[2k], g[2k+1]; col: scratch for the column) and the two scalars
// given, so the single thread that runs it waits on no memory load.
__device__ void arnoldi_update(const Krylov& kr, int s, int k, const double* h1, const double* h2, const double* rot,
                               double* col, int iters, double target) {
    const int m = kr.m;
    double* colg = kr.H + ((long long)s * m + k) * 2 * (m + 1);
    double* hs = kr.hsum + (long long)s * 2 * (m + 1);
    double h2n = 0.0, cnorm = 0.0;
    for (int i = 0; i <= k; ++i) {
        const double re = h1[2 * i] + h2[2 * i], im = h1[2 * i + 1] + h2[2 * i + 1];
        hs[2 * i] = re;
        hs[2 * i + 1] = im;
        col[2 * i] = re;
        col[2 * i + 1] = im;
        h2n += h2[2 * i] * h2[2 * i] + h2[2 * i + 1] * h2[2 * i + 1];
        cnorm += re * re + im * im;
    }
    const double wn2 = h2[2 * (k + 1)];
    const double hn = sqrt(fmax(wn2 - h2n, 0.0));
    cnorm = sqrt(cnorm + hn * hn);
    // previous rotations: [c s; -conj(s) c]
    const double* cs = rot;
    const double* sn = rot + k;
    for (int i = 0; i < k; ++i) {
        const double ar = col[2 * i], ai = col[2 * i + 1], br = col[2 * i + 2], bi = col[2 * i + 3];
        const double c = cs[i], sr = sn[2 * i], si = sn[2 * i + 1];
        col[2 * i] = c * ar + (sr * br - si * bi);
        col[2 * i + 1] = c * ai + (sr * bi + si * br);
        col[2 * i + 2] = -(sr * ar + si * ai) + c * br;
        col[2 * i + 3] = -(sr * ai - si * ar) + c * bi;
    }
    // new rotation zeroing the subdiagonal hn (real, >= 0)
    const double ar = col[2 * k], ai = col[2 * k + 1];
    const double aa = sqrt(ar * ar + ai * ai);
    const double nu = sqrt(aa * aa + hn * hn);
    double c, sr, si, rr, ri;
    if (hn == 0.0) {
        c = 1.0; sr = 0.0; si = 0.0; rr = ar; ri = ai;
    } else if (aa == 0.0) {
        c = 0.0; sr = 1.0; si = 0.0; rr = hn; ri = 0.0;
    } else {
        c = aa / nu;
        sr = (ar / aa) * hn / nu;
        si = (ai / aa) * hn / nu;
        rr = ar * nu / aa;
        ri = ai * nu / aa;
    }
    col[2 * k] = rr;
    col[2 * k + 1] = ri;
    for (int i = 0; i < 2 * (k + 1); ++i) colg[i] = col[i];
    kr.cs[(long long)s * m + k] = c;
    kr.sn[(long long)s * 2 * m + 2 * k] = sr;
    kr.sn[(long long)s * 2 * m + 2 * k + 1] = si;
    double* g = kr.g + (long long)s * 2 * (m + 1);
    const double gr = rot[3 * k], gi = rot[3 * k + 1];
    g[2 * k] = c * gr;
    g[2 * k + 1] = c * gi;
    const double gnr = -(sr * gr + si * gi), gni = -(sr * gi - si * gr);
    g[2 * k + 2] = gnr;
    g[2 * k + 3] = gni;
    const double res = sqrt(gnr * gnr + gni * gni);
    kr.iters[s] = iters + 1;
    kr.hinv[s] = hn > 0.0 ? 1.0 / hn : 0.0;
    if (!isfinite(res) || !isfinite(hn)) {
        kr.err[0] = 1;
        kr.kcount[s] = 0;
        kr.iter_active[s] = 0;
        kr.solve_active[s] = 0;
        return;
    }
    const bool breakdown = hn <= 1e-14 * cnorm;
    if (res <= target || breakdown || k + 1 == m) {
        kr.kcount[s] = k + 1;
        kr.iter_active[s] = 0;
    }
}

// The rotations of the earlier columns and g[2k], g[2k+1] of system si into LDS (whole workgroup).
__device__ void stage_rotations(const Krylov& kr, int si, int k, double* rot) {
    const int m = kr.m;
    for (int u = threadIdx.x; u < 3 * k + 2; u += blockDim.x) {
        if (u < k) rot[u] = kr.cs[(long long)si * m + u];
        else if (u < 3 * k) rot[u] = kr.sn[(long long)si * 2 * m + (u - k)];
        else rot[u] = kr.g[(long long)si * 2 * (m + 1) + 2 * k + (u - 3 * k)];
    }
    __syncthreads();
}

// The nvals sums of a pass over partials part[v * P + t], t in [beg, end), in a fixed order (one wave per
// value), into LDS out (whole workgroup).
__device__ void pass_sums(const double* part, long long P, int beg, int end, int nvals, double* out) {
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63, nw = (int)blockDim.x >> 6;
    for (int v = wv; v < nvals; v += nw) {
        double a = 0.0;
        for (int t = beg + lane; t < end; t += 64) a += part[v * P + t];
        a = wave_sum(a);
        if (lane == 0) out[v] = a;
    }
    __syncthreads();
}

constexpr int kGsGrid = 128;   // workgroups of k_gs (at least one per system)

// Both Gram-Schmidt passes of Arnoldi step k in one launch.  Workgroup b serves system b % S as its
// (b / S)-th workgroup; each reduces the system's first pass (the per-tile partials of the operator
// apply, part1) into LDS in the same fixed order, so all of them take the same decision on the second
// pass.  Without it, the system's first workgroup finishes the Arnoldi step and the others exit.  With
// it, the workgroups form the second pass over the system's chunks (w' = w - sum_l h1_l V_l: partials
// of V_l^H w' and |w'|^2, part2), and the workgroup of the system's last chunk (ticket) reduces them
// and finishes the Arnoldi step.
template <int NV, typename VT>
__global__ __launch_bounds__(kBlock) void k_gs(const Sys* sys, const Chunk* chunks, Krylov kr, int S, int k,
                                              const double* part1, long long P1, const VT* V, long long vstride,
                                              const VT* w, double* part2, int nchunks, long long NT) {
    constexpr int NH = 2 * (kMaxRestart + 1) + 1;
    constexpr int EPT = kChunk / kBlock;
    __shared__ double hh[2][NH], rot[3 * kMaxRestart + 2], col[2 * (kMaxRestart + 1)];
    __shared__ double lds[4 * (2 * NV + 1)];
    __shared__ zd cf[NV];
    __shared__ int flag;
    const int si = blockIdx.x % S, j = blockIdx.x / S, nb = ((int)gridDim.x - si + S - 1) / S;
    if (!kr.iter_active[si]) {
        if (j == 0 && threadIdx.x == 0) kr.reorth[si] = 0;
        return;
    }
    const Sys s = sys[si];
    const int nv = k + 1, nvals = 2 * nv + 1;
    pass_sums(part1, P1, s.tbeg, s.tend, nvals, hh[0]);
    // one classical Gram-Schmidt pass leaves the new vector orthogonal to about eps |w| / |w'|: a second
    // pass when |w'|^2 = |w|^2 - |h1|^2 fell below reorth_theta |w|^2 (theta from rtol, api.hip)
    double hn = 0.0;
    for (int i = 0; i <= k; ++i) hn += hh[0][2 * i] * hh[0][2 * i] + hh[0][2 * i + 1] * hh[0][2 * i + 1];
    const double wn2 = hh[0][2 * nv];
    const bool need = kr.always_reorth || wn2 - hn < kr.reorth_theta * wn2;
    if (!need) {
        if (j != 0) return;
        if (threadIdx.x == 0) {
            kr.reorth[si] = 0;
            for (int i = 0; i <= k; ++i) hh[1][2 * i] = hh[1][2 * i + 1] = 0.0;
            hh[1][2 * nv] = wn2 - hn;
        }
        stage_rotations(kr, si, k, rot);
        if (threadIdx.x == 0) arnoldi_update(kr, si, k, hh[0], hh[1], rot, col, kr.iters[si], kr.target[si]);
        return;
    }
    if (j == 0 && threadIdx.x == 0) kr.reorth[si] = 1;
    if (threadIdx.x < NV) cf[threadIdx.x] = (int)threadIdx.x < nv ? zd{hh[0][2 * threadIdx.x], hh[0][2 * threadIdx.x + 1]}
                                                                  : zd{0.0, 0.0};
    __syncthreads();
    const long long twoN = 2 * s.N;
    for (int ci = s.cbeg + j; ci < s.cend; ci += nb) {
        const Chunk ch = chunks[ci];
        double acc[2 * NV + 1];
#pragma unroll
        for (int i = 0; i < 2 * NV + 1; ++i) acc[i] = 0.0;
        for (int u = 0; u < EPT; ++u) {
            const long long e = (long long)ch.e0 + threadIdx.x + (long long)u * kBlock;
            if (e >= twoN) break;
            const long long gi = elem_index(s, NT, e);
            zd vv[NV];
#pragma unroll
            for (int l = 0; l < NV; ++l) vv[l] = l < nv ? ld<double>(V, l * vstride + gi) : zd{0.0, 0.0};
            zd wv = ld<double>(w, gi);
#pragma unroll
            for (int l = 0; l < NV; ++l) wv = wv - cmul(cf[l], vv[l]);
#pragma unroll
            for (int l = 0; l < NV; ++l) {
                const zd t = cdot(vv[l], wv);
                acc[2 * l] += t.x;
                acc[2 * l + 1] += t.y;
            }
            acc[2 * NV] += abs2(wv);
        }
        block_sum<2 * NV + 1>(acc, lds);
        if (threadIdx.x == 0) {
#pragma unroll
            for (int l = 0; l < NV; ++l)
                if (l < nv) {
                    part2[(2 * l) * (long long)nchunks + ci] = acc[2 * l];
                    part2[(2 * l + 1) * (long long)nchunks + ci] = acc[2 * l + 1];
                }
            part2[(2 * nv) * (long long)nchunks + ci] = acc[2 * NV];
        }
        if (last_of_system(kr.tick_c, si, s.cend - s.cbeg, &flag)) {
            pass_sums(part2, nchunks, s.cbeg, s.cend, nvals, hh[1]);
            stage_rotations(kr, si, k, rot);
            if (threadIdx.x == 0) arnoldi_update(kr, si, k, hh[0], hh[1], rot, col, kr.iters[si], kr.target[si]);
        }
    }
}

__global__ void k_solve_y(Krylov kr, int S) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= S || !kr.solve_active[s]) return;
    const int kc = kr.kcount[s], m = kr.m;
    if (kc <= 0) return;
    const double* g = kr.g + (long long)s * 2 * (m + 1);
    double* y = kr.y + (long long)s * 2 * m;
    for (int i = kc - 1; i >= 0; --i) {
        double tr = g[2 * i], ti = g[2 * i + 1];
        for (int l = i + 1; l < kc; ++l) {
            const double* col = kr.H + ((long long)s * m + l) * 2 * (m + 1);
            const double hr = col[2 * i], hi = col[2 * i + 1];
            tr -= hr * y[2 * l] - hi * y[2 * l + 1];
            ti -= hr * y[2 * l + 1] + hi * y[2 * l];
        }
        const double* cc = kr.H + ((long long)s * m + i) * 2 * (m + 1);
        const double dr = cc[2 * i], di = cc[2 * i + 1];
        const double den = dr * dr + di * di;
        y[2 * i] = den > 0.0 ? (tr * dr + ti * di) / den : 0.0;
        y[2 * i + 1] = den > 0.0 ? (ti * dr - tr * di) / den : 0.0;
    }
}

// ------------------------------------------------------------------------------------------
// energy, its gradient, adjoint pieces
// ------------------------------------------------------------------------------------------
// per tile: E0 = sum 2 Re(zeta^H G eta) - zeta^H M zeta (= eta^H G M^{-1} G eta to second order
// in the error of zeta); E1 = sum w f^s(eta) on the amplitude-0 tiles of each instance.
template <int DIM, int TY>
__global__ __launch_bounds__(kBlock) void k_energy(const Sys* sys, const Tile* tiles, const Terms T, const zd* eta,
                                                  const zd* zeta, double* part, int ntiles) {
    __shared__ double lds[8];
    const int* mask = nullptr;
    TILE_PROLOGUE();
    double acc[2] = {0.0, 0.0};
    FOR_ROWS(TY) {
        Nbr<DIM> n;
        make_nbr<DIM>(s, x, y, pz, n);
        zd Me, Ke, Te, Mz, Kz, Tz;
        stencil<DIM, true, true, double>([&](int a, int b, int c) { return eta[s.off + nb_index<DIM>(n, a, b, c)]; },
                                         s.h, s.kv[0], s.kv[1], s.kv[2], Me, Ke, Te);
        stencil<DIM, false, false, double>(
            [&](int a, int b, int c) { return zeta[s.off + nb_index<DIM>(n, a, b, c)]; }, s.h, 0.0, 0.0, 0.0, Mz,
            Kz, Tz);
        const long long il = nb_index<DIM>(n, 1, 1, 1);
        const zd zc = zeta[s.off + il];
        acc[0] += 2.0 * cdot(zc, gop(Ke, Te)).x - cdot(zc, Mz).x;
        if (s.j == 0) {
            zd e[kMaxJ];
            for (int l = 0; l < T.J; ++l) e[l] = eta[s.off + l * s.N + il];
            acc[1] += s.w * bulk_f(T, s, e);
        }
    }
    block_sum<2>(acc, lds);
    if (threadIdx.x == 0) {
        part[kE0 * (long long)ntiles + blockIdx.x] = acc[0];
        part[kE1 * (long long)ntiles + blockIdx.x] = acc[1];
    }
}

// grad_j = 2 (w F^s_j(eta) + G_j zeta_j) (planar output); partial of dE/dDeltaB = sum w A/(2 a0).
template <int DIM, int TY>
__global__ __launch_bounds__(kBlock) void k_energy_grad(const Sys* sys, const Tile* tiles, const Terms T,
                                                       const zd* eta, const zd* zeta, double* const* grad_tab,
                                                       double* part, int ntiles) {
    __shared__ double lds[4];
    const int* mask = nullptr;
    TILE_PROLOGUE();
    double* g = grad_tab[s.inst] + (long long)s.j * 2 * s.N;
    double acc[1] = {0.0};
    FOR_ROWS(TY) {
        Nbr<DIM> n;
        make_nbr<DIM>(s, x, y, pz, n);
        zd Mz, Kz, Tz;
        stencil<DIM, true, true, double>([&](int a, int b, int c) { return zeta[s.off + nb_index<DIM>(n, a, b, c)]; },
                                         s.h, s.kv[0], s.kv[1], s.kv[2], Mz, Kz, Tz);
        const long long il = nb_index<DIM>(n, 1, 1, 1);
        const long long i0 = s.off - (long long)s.j * s.N;     // amplitude 0 of this instance
        zd e[kMaxJ], h[kMaxJ];
        double A = 0.0;
        for (int l = 0; l < T.J; ++l) {
            e[l] = eta[i0 + l * s.N + il];
            A += abs2(e[l]);
        }
        double d;
        bulk_h(T, s, e, d, h);
        const zd F = d * e[s.j] + h[s.j];
        const zd gv = 2.0 * (s.w * F + gop(Kz, Tz));
        g[il] = gv.x;
        g[s.N + il] = gv.y;
        if (s.j == 0) acc[0] += s.w * 2.0 * A / (2.0 * s.a0);
    }
    block_sum<1>(acc, lds);
    if (threadIdx.x == 0) part[kE1 * (long long)ntiles + blockIdx.x] = acc[0];
}

// Local rotation (Eq. (14)-(15)) and target mesh size (Eq. (16)-(17)) at every node of an instance
// (launched on the amplitude-0 tiles).  Phase gradients from central differences of eta_j,
// du/dx_b by least squares over the amplitudes carrying a phase.
template <int DIM, int TY>
__global__ __launch_bounds__(kBlock) void k_rotation(const Sys* sys, const Tile* tiles, const Terms T, const zd* eta,
                                                    double* const* omega_tab, double* const* h_tab, RefineArgs ra) {
    const int* mask = nullptr;
    TILE_PROLOGUE();
    if (s.j != 0) return;
    double* om = omega_tab[s.inst];
    double* hh = h_tab ? h_tab[s.inst] : nullptr;
    const int J = T.J;
    FOR_ROWS(TY) {
        Nbr<DIM> n;
        make_nbr<DIM>(s, x, y, pz, n);
        const long long il = nb_index<DIM>(n, 1, 1, 1);
        double KtK[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
        double rhs[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};     // rhs[b][a'] = sum_j k_{j,a'} d theta_j/dx_b
        double Ac = 0.0, gA[3] = {0, 0, 0};
        for (int l = 0; l < J; ++l) {
            const Sys& sl = sys[tile.sys + l];
            const zd* e = eta + sl.off;
            const zd c = e[il];
            const double m2 = abs2(c);
            Ac += 2.0 * m2;
            const bool ok = m2 > ra.tiny;
            for (int b = 0; b < DIM; ++b) {
                const long long ip = b == 0 ? nb_index<DIM>(n, 2, 1, 1) : (b == 1 ? nb_index<DIM>(n, 1, 2, 1) : nb_index<DIM>(n, 1, 1, 2));
                const long long im = b == 0 ? nb_index<DIM>(n, 0, 1, 1) : (b == 1 ? nb_index<DIM>(n, 1, 0, 1) : nb_index<DIM>(n, 1, 1, 0));
                const zd ep = e[ip], em = e[im];
                gA[b] += 2.0 * (abs2(ep) - abs2(em)) / (2.0 * s.h);
                if (ok) {
                    const zd de = (0.5 / s.h) * (ep - em);
                    const double dth = cdot(c, de).y / m2;
                    for (int a = 0; a < DIM; ++a) rhs[b][a] += sl.kv[a] * dth;
                }
            }
            if (ok)
                for (int a = 0; a < DIM; ++a)
                    for (int a2 = 0; a2 < DIM; ++a2) KtK[a][a2] += sl.kv[a] * sl.kv[a2];
        }
        // invert the symmetric DIM x DIM matrix
        double inv[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
        double det, tr = 0.0;
        for (int a = 0; a < DIM; ++a) tr += KtK[a][a];
        if constexpr (DIM == 2) {
            det = KtK[0][0] * KtK[1][1] - KtK[0][1] * KtK[1][0];
            inv[0][0] = KtK[1][1];
            inv[1][1] = KtK[0][0];
            inv[0][1] = -KtK[0][1];
            inv[1][0] = -KtK[1][0];
        } else {
            inv[0][0] = KtK[1][1] * KtK[2][2] - KtK[1][2] * KtK[2][1];
            inv[0][1] = KtK[0][2] * KtK[2][1] - KtK[0][1] * KtK[2][2];
            inv[0][2] = KtK[0][1] * KtK[1][2] - KtK[0][2] * KtK[1][1];
            inv[1][0] = KtK[1][2] * KtK[2][0] - KtK[1][0] * KtK[2][2];
            inv[1][1] = KtK[0][0] * KtK[2][2] - KtK[0][2] * KtK[2][0];
            inv[1][2] = KtK[0][2] * KtK[1][0] - KtK[0][0] * KtK[1][2];
            inv[2][0] = KtK[1][0] * KtK[2][1] - KtK[1][1] * KtK[2][0];
            inv[2][1] = KtK[0][1] * KtK[2][0] - KtK[0][0] * KtK[2][1];
            inv[2][2] = KtK[0][0] * KtK[1][1] - KtK[0][1] * KtK[1][0];
            det = KtK[0][0] * inv[0][0] + KtK[0][1] * inv[1][0] + KtK[0][2] * inv[2][0];
        }
        const bool solvable = tr > 0.0 && det > 1e-12 * pow(tr / DIM, (double)DIM);
        double Gu[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};         // Gu[a][b] = du_a/dx_b
        if (solvable)
            for (int a = 0; a < DIM; ++a)
                for (int b = 0; b < DIM; ++b) {
                    double v = 0.0;
                    for (int a2 = 0; a2 < DIM; ++a2) v += inv[a][a2] * rhs[b][a2];
                    Gu[a][b] = v / det;
                }
        double omax;
        if constexpr (DIM == 2) {
            const double w = 0.5 * (Gu[0][1] - Gu[1][0]);
            om[il] = w;
            omax = fabs(w);
        } else {
            const double w0 = 0.5 * (Gu[1][2] - Gu[2][1]), w1 = 0.5 * (Gu[2][0] - Gu[0][2]), w2 = 0.5 * (Gu[0][1] - Gu[1][0]);
            om[il] = w0;
            om[s.N + il] = w1;
            om[2 * s.N + il] = w2;
            omax = fmax(fabs(w0), fmax(fabs(w1), fabs(w2)));
        }
        if (hh) {
            double g2 = 0.0;
            for (int b = 0; b < DIM; ++b) g2 += gA[b] * gA[b];
            const double theta = asin(fmin(omax, 1.0));
            const double lam = theta > 0.0 ? 2.0 * 3.14159265358979323846 / (2.0 * ra.kmax * sin(0.5 * theta)) : INFINITY;
            const double hamp = lam / ra.nwl;
            hh[il] = sqrt(g2) >= ra.eps ? ra.hint : (Ac > ra.Amin ? fmin(fmax(hamp, ra.hint), ra.hmax) : ra.hmax);
        }
    }
}

// adjoint right-hand side [0 ; lam_j]
template <int DIM, int TY>
__global__ __launch_bounds__(kBlock) void k_adjoint_rhs(const Sys* sys, const Tile* tiles, double* const* lam_tab,
                                                       zd* B, long long NT) {
    const int* mask = nullptr;
    TILE_PROLOGUE();
    const double* lam = lam_tab[s.inst] + (long long)s.j * 2 * s.N;
    FOR_ROWS(TY) {
        const long long i = ((long long)pz * s.ny + y) * s.nx + x;
        B[s.off + i] = zd{0.0, 0.0};
        B[NT + s.off + i] = zd{lam[i], lam[s.N + i]};
    }
}

// lam_before_l = M mu_l / dt + nodal adjoint of -kappa_j w h_j(eta) and of kappa_j w diag(d(eta)) eta^m_j.
// mu_j = eta part of Y = A_j^{-1} [0; lam_j] (Sigma leaves the eta part unchanged).
// Launched on amplitude-0 tiles; computes every amplitude of the instance at the node.
template <int DIM, int TY>
__global__ __launch_bounds__(kBlock) void k_adjoint_out(const Sys* sys, const Tile* tiles, const Terms T, const zd* Y,
                                                       const zd* eta_prev, double* const* eta_new_tab,
                                                       double* const* lam_out_tab, double* part, int ntiles,
                                                       long long NT) {
    __shared__ double lds[4];
    const int* mask = nullptr;
    TILE_PROLOGUE();
    double acc[1] = {0.0};
    if (s.j == 0) {
        const double* en = eta_new_tab[s.inst];
        double* lo = lam_out_tab[s.inst];
        const int J = T.J;
        FOR_ROWS(TY) {
            Nbr<DIM> n;
            make_nbr<DIM>(s, x, y, pz, n);
            const long long il = nb_index<DIM>(n, 1, 1, 1);
            zd ep[kMaxJ], nu[kMaxJ], gr[kMaxJ];
            double C = 0.0;
            for (int l = 0; l < J; ++l) {
                const Sys& sl = sys[tile.sys + l];
                const zd* mu = Y + NT;
                zd Mm, Km, Tm;
                stencil<DIM, false, false, double>(
                    [&](int a, int b, int c) { return mu[sl.off + nb_index<DIM>(n, a, b, c)]; }, s.h, 0.0, 0.0, 0.0,
                    Mm, Km, Tm);
                gr[l] = s.inv_dt * Mm;
                const zd muc = mu[sl.off + il];
                ep[l] = eta_prev[sl.off + il];
                nu[l] = (-sl.kappa * s.w) * muc;
                const zd enl = zd{en[(long long)l * 2 * s.N + il], en[(long long)l * 2 * s.N + s.N + il]};
                C += sl.kappa * s.w * cdot(muc, enl).x;
            }
            // pair term h_j += -4 (a2/a0) eta_j^2 eta_j^*
            const double c4 = 4.0 * s.a2 / s.a0;
            for (int l = 0; l < J; ++l) {
                gr[l] = gr[l] - (2.0 * c4 * abs2(ep[l])) * nu[l] - c4 * cmul(cmul(ep[l], ep[l]), cconj(nu[l]));
            }
            // resonant terms c (T + T^*)
            for (int t = 0; t < T.n; ++t) {
                const double c = term_coef(T, t, s);
                const int ord = T.order[t];
                for (int q = 0; q < ord; ++q) {
                    const zd nq = nu[T.idx[t][q]];
                    const bool direct = T.cj[t][q];   // h_{idx q} += c prod_{r != q} u_r  (else its conjugate)
                    for (int r = 0; r < ord; ++r) {
                        if (r == q) continue;
                        zd a{c, 0.0};
                        for (int r2 = 0; r2 < ord; ++r2)
                            if (r2 != q && r2 != r) {
                                const zd u = factor(T, t, r2, ep);
                                a = cmul(a, direct ? u : cconj(u));
                            }
                        const int l = T.idx[t][r];
                        // the factor r of the contribution is eta_l when (direct and not conjugated) or
                        // (not direct and conjugated); otherwise it is eta_l^*
                        const bool is_eta = direct ? (T.cj[t][r] == 0) : (T.cj[t][r] != 0);
                        gr[l] = gr[l] + (is_eta ? cmul(cconj(a), nq) : cmul(cconj(nq), a));
                    }
                }
            }
            // d = 2 a1/a0 + 8 (a2/a0) sum |eta|^2 enters A as kappa_j w d eta^m_j
            for (int l = 0; l < J; ++l) {
                gr[l] = gr[l] - (16.0 * s.a2 / s.a0 * C) * ep[l];
                lo[(long long)l * 2 * s.N + il] = gr[l].x;
                lo[(long long)l * 2 * s.N + s.N + il] = gr[l].y;
            }
            acc[0] += -C / s.a0;
        }
    }
    block_sum<1>(acc, lds);
    if (threadIdx.x == 0) part[kE1 * (long long)ntiles + blockIdx.x] = acc[0];
}

// ------------------------------------------------------------------------------------------
// launch plumbing
// ------------------------------------------------------------------------------------------
static const char* kNames[KID_COUNT] = {"pcg_spmv", "pcg_update", "pcg_init", "pc_final", "apply", "residual",
                                        "gs",       "proj_final", "xupdate",  "reduce",   "small", "other",
                                        "cheb",     "extrapolate", "rhs",  "mg",    "mass"};
const char* kernel_name(int kid) { return (kid >= 0 && kid < KID_COUNT) ? kNames[kid] : (kid == KID_ALL ? "all" : "none"); }
int kernel_id(const char* name) {
    if (!name) return KID_NONE;
    if (name[0] == 'a' && name[1] == 'l' && name[2] == 'l' && name[3] == 0) return KID_ALL;
    for (int i = 0; i < KID_COUNT; ++i) {
        const char* a = kNames[i];
        const char* b = name;
        while (*a && *a == *b) ++a, ++b;
        if (*a == 0 && *b == 0) return i;
    }
    return KID_NONE;
}

// Share of the batch's nodes that belong to the systems a masked launch works on (1 without a mask):
// converged systems are skipped by the kernels and move no bytes.
__global__ __launch_bounds__(kBlock) void k_active_frac(const Sys* sys, int S, const int* mask, double* out) {
    __shared__ double lds[2 * (kBlock / 64)];
    double acc[2] = {0.0, 0.0};
    for (int s = threadIdx.x; s < S; s += kBlock) {
        const double n = (double)sys[s].N;
        acc[0] += (!mask || mask[s]) ? n : 0.0;
        acc[1] += n;
    }
    block_sum<2>(acc, lds);
    if (threadIdx.x == 0) *out = acc[1] > 0.0 ? acc[0] / acc[1] : 0.0;
}

void launch_active_frac(const Sys* sys, int S, const int* mask, double* out, hipStream_t st) {
    hipLaunchKernelGGL(k_active_frac, dim3(1), dim3(kBlock), 0, st, sys, S, mask, out);
}

void launch_state_in(const Dev& d, double* const* eta_tab, double* const* zeta_tab, zd* X, hipStream_t st) {
    ProbeScope ps(d, KID_OTHER, st);
    dispatch(d, [&](auto D, auto TY) {
        hipLaunchKernelGGL((k_state_in<D(), TY()>), TILE_GRID, d.sys, d.tiles, nullptr, eta_tab, zeta_tab, X, d.NT);
    });
}
void launch_state_out(const Dev& d, const zd* X, double* const* eta_tab, double* const* zeta_tab, hipStream_t st) {
    dispatch(d, [&](auto D, auto TY) {
        hipLaunchKernelGGL((k_state_out<D(), TY()>), TILE_GRID, d.sys, d.tiles, nullptr, X, eta_tab, zeta_tab, d.NT);
    });
}
void launch_planar_in(const Dev& d, double* const* tab, zd* half, hipStream_t st) {
    dispatch(d, [&](auto D, auto TY) {
        hipLaunchKernelGGL((k_planar<D(), TY(), true>), TILE_GRID, d.sys, d.tiles, nullptr, tab, half);
    });
}
void launch_planar_out(const Dev& d, const zd* half, double* const* tab, hipStream_t st) {
    dispatch(d, [&](auto D, auto TY) {
        hipLaunchKernelGGL((k_planar<D(), TY(), false>), TILE_GRID, d.sys, d.tiles, nullptr, tab,
                           const_cast<zd*>(half));
    });
}
void launch_fill_zero(zd* p, long long n, hipStream_t st) {
    if (n <= 0) return;
    long long blocks = (n + kBlock - 1) / kBlock;
    if (blocks > 8192) blocks = 8192;
    hipLaunchKernelGGL(k_fill_zero, dim3((unsigned)blocks), dim3(kBlock), 0, st, p, n);
}
__global__ __launch_bounds__(kBlock) void k_widen(const zf* in, zd* out, long long n) {
    for (long long i = blockIdx.x * (long long)kBlock + threadIdx.x; i < n; i += (long long)gridDim.x * kBlock)
        out[i] = zd{(double)in[i].x, (double)in[i].y};
}
__global__ __launch_bounds__(kBlock) void k_narrow(const zd* in, zf* out, long long n) {
    for (long long i = blockIdx.x * (long long)kBlock + threadIdx.x; i < n; i += (long long)gridDim.x * kBlock)
        out[i] = zf{(float)in[i].x, (float)in[i].y};
}
// Initial guess from the kept states h_1 (newest) .. h_K: the polynomial through x and the last
// `order` kept states, evaluated one step ahead (order 0: x; 1: 2x - h1; 2: 3x - 3h1 + h2;
// 3: 4x - 6h1 + 4h2 - h3), written to X0.  With keep != null the state x is also copied there (the
// oldest kept state's buffer, possibly h_order itself: each element is read before it is written); the
// guess may then overwrite X in place.  With keep = null, X0 is a buffer of its own and X is only read
// (the caller keeps X's buffer as the newest state).
template <int ORDER>
__global__ __launch_bounds__(kBlock) void k_extrapolate(const zd* X, const zd* h1, const zd* h2, const zd* h3,
                                                       zd* X0, zd* keep, long long n) {
    for (long long i = blockIdx.x * (long long)kBlock + threadIdx.x; i < n; i += (long long)gridDim.x * kBlock) {
        const zd x = X[i];
        zd g = x;
        if constexpr (ORDER == 1) g = x + (x - h1[i]);
        else if constexpr (ORDER == 2) g = h2[i] + 3.0 * (x - h1[i]);
        else if constexpr (ORDER == 3) g = 4.0 * (x + h2[i]) - (6.0 * h1[i] + h3[i]);
        if (keep) keep[i] = x;
        X0[i] = g;
    }
}
void launch_extrapolate(const Dev& d, const zd* X, const zd* const* h, zd* X0, zd* keep, int order, hipStream_t st) {
    const long long n = 2 * d.NT;
    // reads x and `order` kept states, writes the guess (and the kept copy)
    ProbeScope ps(d, KID_EXTRAP, st, (double)n * sizeof(zd) * (order + 2 + (keep ? 1 : 0)));
    long long blocks = (n + kBlock - 1) / kBlock;
    if (blocks > 65536) blocks = 65536;
    auto go = [&](auto oc) {
        hipLaunchKernelGGL((k_extrapolate<decltype(oc)::value>), dim3((unsigned)blocks), dim3(kBlock), 0, st, X, h[0],
                           h[1], h[2], X0, keep, n);
    };
    switch (order) {
        case 1: go(std::integral_constant<int, 1>{}); break;
        case 2: go(std::integral_constant<int, 2>{}); break;
        case 3: go(std::integral_constant<int, 3>{}); break;
        default: go(std::integral_constant<int, 0>{}); break;
    }
}

void launch_widen(const zf* in, zd* out, long long n, hipStream_t st) {
    if (n <= 0) return;
    long long blocks = (n + kBlock - 1) / kBlock;
    if (blocks > 8192) blocks = 8192;
    hipLaunchKernelGGL(k_widen, dim3((unsigned)blocks), dim3(kBlock), 0, st, in, out, n);
}
void launch_narrow(const zd* in, zf* out, long long n, hipStream_t st) {
    if (n <= 0) return;
    long long blocks = (n + kBlock - 1) / kBlock;
    if (blocks > 8192) blocks = 8192;
    hipLaunchKernelGGL(k_narrow, dim3((unsigned)blocks), dim3(kBlock), 0, st, in, out, n);
}
void launch_rhs_base(const Dev& d, const zd* Xeta, double* const* src_tab, zd* BB, hipStream_t st) {
    // reads eta (and s), writes BB
    ProbeScope ps(d, KID_RHS, st, (double)d.NT * sizeof(zd) * (2.0 + (src_tab ? 1.0 : 0.0)));
    dispatch(d, [&](auto D, auto TY) {
        if constexpr (D() == 3) {
            if (src_tab)
                hipLaunchKernelGGL((k_rhs_base3d<TY(), true>), TILE_GRID, d.sys, d.tiles, Xeta, src_tab, BB);
            else
                hipLaunchKernelGGL((k_rhs_base3d<TY(), false>), TILE_GRID, d.sys, d.tiles, Xeta, src_tab, BB);
        } else {
            hipLaunchKernelGGL((k_rhs_base<D(), TY()>), TILE_GRID, d.sys, d.tiles, nullptr, Xeta, src_tab, BB);
        }
    });
}
// amplitude slots of the register-resident nonlinearity: 3 (triangular), 6 (bcc), else 8
template <typename F>
static void dispatch_jm(int J, F&& f) {
    if (J == 3) f(std::integral_constant<int, 3>{});
    else if (J == 6) f(std::integral_constant<int, 6>{});
    else f(std::integral_constant<int, kMaxJ>{});
}
void launch_nonlinear(const Dev& d, const zd* eta_half, const zd* BB, double* dnode, zd* B, hipStream_t st) {
    // reads eta and BB, writes B (both halves) and d
    ProbeScope ps(d, KID_RHS, st, (double)d.NT * sizeof(zd) * 4.0 + (double)d.NT * 8.0 / d.J);
    dispatch(d, [&](auto D, auto TY) {
        dispatch_jm(d.J, [&](auto JM) {
            hipLaunchKernelGGL((k_nonlinear<D(), TY(), JM()>), TILE_GRID, d.sys, d.tiles, d.terms, eta_half, BB,
                               dnode, B, d.NT);
        });
    });
}
void launch_rhs_nonlinear(const Dev& d, const zd* eta_half, double* const* src_tab, double* dnode, zd* B,
                          hipStream_t st) {
    // reads eta (each amplitude once; the other amplitudes of a node come through L2), writes B (both
    // halves) and d (per instance node); a source adds one read of s
    ProbeScope ps(d, KID_RHS, st, (double)d.NT * (sizeof(zd) * (3.0 + (src_tab ? 1.0 : 0.0)) + 8.0 / d.J));
    dispatch(d, [&](auto D, auto TY) {
        dispatch_jm(d.J, [&](auto JM) {
            hipLaunchKernelGGL((k_rhs_nonlinear<D(), TY(), JM()>), TILE_GRID, d.sys, d.tiles, d.terms, eta_half,
                               src_tab, dnode, B, d.NT);
        });
    });
}
template <int DIM, int TY, typename T, int OP>
static void cg_iterations(const Dev& d, cx<T>* xv, cx<T>* r, cx<T>* p0, cx<T>* p1, cx<T>* q, double* part, int n,
                          const int* mask, hipStream_t st) {
    cx<T>* P[2] = {p0, p1};
    for (int it = 0; it < n; ++it) {
        {
            // algorithmic bytes: FIRST reads p, writes q; otherwise reads r, p and writes p, q
            const double nb = (double)d.NT * sizeof(cx<T>) * (it == 0 ? 2.0 : 4.0);
            ProbeScope ps(d, KID_PCG_SPMV, st, nb);
            if (it == 0)
                hipLaunchKernelGGL((k_cg_spmv<DIM, TY, T, OP, true>), TILE_GRID, d.sys, d.tiles, mask, r, p0, p0, q,
                                   part, d.ntiles, it);
            else
                hipLaunchKernelGGL((k_cg_spmv<DIM, TY, T, OP, false>), TILE_GRID, d.sys, d.tiles, mask, r,
                                   P[(it - 1) & 1], P[it & 1], q, part, d.ntiles, it);
        }
        const bool first = it == 0, last = it == n - 1;
        // reads p (+x unless first, + r, q unless last), writes x (+ r unless last)
        const double nb = (double)d.NT * sizeof(cx<T>) * (2.0 + (first ? 0.0 : 1.0) + (last ? 0.0 : 3.0));
        ProbeScope ps(d, KID_PCG_UPDATE, st, nb);
        cx<T>* pv = P[it & 1];
        if (first && last)
            hipLaunchKernelGGL((k_cg_update<DIM, TY, T, OP, true, true>), TILE_GRID, d.sys, d.tiles, mask, xv, r, pv,
                               q, part, d.ntiles, it);
        else if (first)
            hipLaunchKernelGGL((k_cg_update<DIM, TY, T, OP, true, false>), TILE_GRID, d.sys, d.tiles, mask, xv, r,
                               pv, q, part, d.ntiles, it);
        else if (last)
            hipLaunchKernelGGL((k_cg_update<DIM, TY, T, OP, false, true>), TILE_GRID, d.sys, d.tiles, mask, xv, r,
                               pv, q, part, d.ntiles, it);
        else
            hipLaunchKernelGGL((k_cg_update<DIM, TY, T, OP, false, false>), TILE_GRID, d.sys, d.tiles, mask, xv, r,
                               pv, q, part, d.ntiles, it);
    }
}

template <typename T>
void launch_precond(const Dev& d, const cx<T>* v, cx<T>* z, cx<T>* x1, cx<T>* x2, cx<T>* r, cx<T>* p0, cx<T>* p1,
                    cx<T>* q, double* part, int mass_iters, int diff_iters, int mass_sep, const int* mask,
                    hipStream_t st) {
    dispatch(d, [&](auto D, auto TY) {
        constexpr int DIM = D(), TYv = TY();
        // step 1: beta1' ~ M^{-1} beta1
        if (mass_sep > 0) {
            launch_mass_sep<T>(d, mass_sep, v, x1, mask, st);
        } else {
            {
                ProbeScope ps(d, KID_PCG_INIT, st);
                hipLaunchKernelGGL((k_cg_init_copy<DIM, TYv, T>), TILE_GRID, d.sys, d.tiles, mask, v, r, p0, part,
                                   d.ntiles);
            }
            cg_iterations<DIM, TYv, T, 0>(d, x1, r, p0, p1, q, part, mass_iters, mask, st);
        }
        // step 2: beta2' ~ L^{-1} (beta2 - kappa G beta1')
        {
            ProbeScope ps(d, KID_PCG_INIT, st);
            hipLaunchKernelGGL((k_cg_init_g<DIM, TYv, T>), TILE_GRID, d.sys, d.tiles, mask, v, x1, r, p0, part,
                               d.ntiles, d.NT);
        }
        cg_iterations<DIM, TYv, T, 1>(d, x2, r, p0, p1, q, part, diff_iters, mask, st);
        // step 3: chi2 ~ L^{-1} M beta2'  (written straight into the eta part of z)
        {
            ProbeScope ps(d, KID_PCG_INIT, st);
            hipLaunchKernelGGL((k_cg_init_m<DIM, TYv, T, false>), TILE_GRID, d.sys, d.tiles, mask, x2, r, p0, part,
                               d.ntiles);
        }
        cg_iterations<DIM, TYv, T, 1>(d, z + d.NT, r, p0, p1, q, part, diff_iters, mask, st);
        // step 4
        ProbeScope ps(d, KID_PC_FINAL, st);
        hipLaunchKernelGGL((k_pc_final<DIM, TYv, T>), TILE_GRID, d.sys, d.tiles, mask, x1, x2, z, d.NT);
    });
}
template void launch_precond<double>(const Dev&, const zd*, zd*, zd*, zd*, zd*, zd*, zd*, zd*, double*, int, int,
                                     int, const int*, hipStream_t);
template void launch_precond<float>(const Dev&, const zf*, zf*, zf*, zf*, zf*, zf*, zf*, zf*, double*, int, int,
                                    int, const int*, hipStream_t);

// stage launch of the Chebyshev inner solves: z-marching kernels for the stencil stages in 3D
template <int DIM, int TY, typename T, int STAGE>
static void cb_init_launch(const Dev& d, const int* mask, const cx<T>* v, const cx<T>* src, cx<T>* r, cx<T>* dd,
                           cx<T>* xv, hipStream_t st) {
    if constexpr (DIM == 3 && STAGE != 0)
        hipLaunchKernelGGL((k_cb_init3d<TY / 4, 4, T, STAGE>), TILE_GRID, d.sys, d.tiles, mask, v, src, r, dd, xv,
                           d.NT);
    else
        hipLaunchKernelGGL((k_cb_init<DIM, TY, T, STAGE>), TILE_GRID, d.sys, d.tiles, mask, v, src, r, dd, xv, d.NT);
}

template <int DIM, int TYv, typename T, int OP>
static void cb_iterations(const Dev& d, int its, cx<T>* d0, cx<T>* d1, cx<T>* r, cx<T>* xv, const int* mask,
                          hipStream_t st) {
    cx<T>* D[2] = {d0, d1};
    for (int j = 1; j < its; ++j) {
        ProbeScope ps(d, KID_CHEB, st, (double)d.NT * sizeof(cx<T>) * (j == its - 1 ? 3.0 : 6.0), mask);
        if constexpr (DIM == 3) {
            if (j == its - 1)
                hipLaunchKernelGGL((k_cb_iter3d<TYv, T, OP, true>), TILE_GRID, d.sys, d.tiles, mask, j,
                                   D[(j - 1) & 1], D[j & 1], r, xv);
            else
                hipLaunchKernelGGL((k_cb_iter3d<TYv, T, OP, false>), TILE_GRID, d.sys, d.tiles, mask, j,
                                   D[(j - 1) & 1], D[j & 1], r, xv);
        } else {
            if (j == its - 1)
                hipLaunchKernelGGL((k_cb_iter<DIM, TYv, T, OP, true>), TILE_GRID, d.sys, d.tiles, mask, j,
                                   D[(j - 1) & 1], D[j & 1], r, xv);
            else
                hipLaunchKernelGGL((k_cb_iter<DIM, TYv, T, OP, false>), TILE_GRID, d.sys, d.tiles, mask, j,
                                   D[(j - 1) & 1], D[j & 1], r, xv);
        }
    }
}

// 3D Chebyshev iterations j0 .. its-1 of one inner solve; with x1 and x2 set, the last one also does
// step 4 of the preconditioner (k_cb_iter3d FINAL).
template <int TYv, typename T, int OP>
static void cb_iterations3d(const Dev& d, int j0, int its, cx<T>* d0, cx<T>* d1, cx<T>* r, cx<T>* xv,
                            const cx<T>* x1, const cx<T>* x2, cx<T>* zz, const int* mask, hipStream_t st) {
    cx<T>* D[2] = {d0, d1};
    for (int j = j0; j < its; ++j) {
        const bool last = j == its - 1;
        ProbeScope ps(d, KID_CHEB, st, (double)d.NT * sizeof(cx<T>) * (last ? (x1 ? 6.0 : 3.0) : 6.0), mask);
        if (last && x1)
            hipLaunchKernelGGL((k_cb_iter3d<TYv, T, OP, true, true>), TILE_GRID, d.sys, d.tiles, mask, j,
                               D[(j - 1) & 1], D[j & 1], r, xv, x1, x2, zz);
        else if (last)
            hipLaunchKernelGGL((k_cb_iter3d<TYv, T, OP, true>), TILE_GRID, d.sys, d.tiles, mask, j, D[(j - 1) & 1],
                               D[j & 1], r, xv, nullptr, nullptr, nullptr);
        else
            hipLaunchKernelGGL((k_cb_iter3d<TYv, T, OP, false>), TILE_GRID, d.sys, d.tiles, mask, j,
                               D[(j - 1) & 1], D[j & 1], r, xv, nullptr, nullptr, nullptr);
    }
}

// Iterations 1 .. its - 1 of a three-term Chebyshev solve for L (3D) after the start wrote b: x_1 = s b is
// formed where needed (j = 1, 2), x_j (j >= 2) in A or B by the parity of j, the last iterate into out (with
// x1, x2, zz: step 4 as well).
template <int TYv, typename T>
static void cx_iterations3d(const Dev& d, int its, cx<T>* A, cx<T>* B, const cx<T>* b, cx<T>* out, const cx<T>* x1,
                            const cx<T>* x2, cx<T>* zz, const int* mask, hipStream_t st) {
    for (int j = 1; j < its; ++j) {
        const bool last = j == its - 1, first = j == 1, prevb = j == 2, fin = last && zz;
        cx<T>* xk = ((j - 1) & 1) ? B : A;
        cx<T>* xkm1 = (j & 1) ? B : A;
        cx<T>* xo = last ? out : xkm1;
        // b (and at j = 1 x_1 = s b from it), x_j, x_{j-1} unless formed from b, x_{j+1}; step 4: x1, x2, z_zeta
        const double vecs = (first ? 2.0 : prevb ? 3.0 : 4.0) + (fin ? 3.0 : 0.0);
        ProbeScope ps(d, KID_CHEB, st, (double)d.NT * sizeof(cx<T>) * vecs, mask, true);
        auto go = [&](auto f, auto p, auto fn) {
            brick_depth(d, [&](auto bz) {
                ps.launch(k_cx_iter3d<decltype(bz)::value, kMassBY, T, decltype(f)::value, decltype(p)::value,
                                      decltype(fn)::value>,
                          dim3(d.nmtiles), dim3(kMassThreads), d.sys, d.mtiles, mask, j, (const cx<T>*)xk,
                          (const cx<T>*)xkm1, b, xo, x1, x2, zz);
            });
        };
        using TT = std::true_type;
        using FF = std::false_type;
        if (fin) {
            if (first) go(TT{}, FF{}, TT{});
            else if (prevb) go(FF{}, TT{}, TT{});
            else go(FF{}, FF{}, TT{});
        } else {
            if (first) go(TT{}, FF{}, FF{});
            else if (prevb) go(FF{}, TT{}, FF{});
            else go(FF{}, FF{}, FF{});
        }
    }
}

template <typename T>
void launch_precond_cheb_unfused(const Dev& d, const cx<T>* v, cx<T>* z, cx<T>* x1, cx<T>* x2, cx<T>* r, cx<T>* d0,
                                 cx<T>* d1, int mass_iters, int diff_iters, int mass_sep, const int* mask,
                                 hipStream_t st) {
    dispatch(d, [&](auto D, auto TY) {
        constexpr int DIM = D(), TYv = TY();
        if constexpr (DIM == 3) {
            // step 1: the separable mass inverse, or the initialisation fused with the first iteration
            if (mass_sep > 0) {
                launch_mass_sep<T>(d, mass_sep, v, x1, mask, st);
            } else if (mass_iters >= 2) {
                ProbeScope ps(d, KID_CHEB, st, (double)d.NT * (mass_iters == 2 ? 2.0 : 4.0) * sizeof(cx<T>), mask);
                if (mass_iters == 2)
                    hipLaunchKernelGGL((k_cb_first3d<TYv, T, true>), TILE_GRID, d.sys, d.tiles, mask, v, d1, r, x1);
                else
                    hipLaunchKernelGGL((k_cb_first3d<TYv, T, false>), TILE_GRID, d.sys, d.tiles, mask, v, d1, r, x1);
            } else {
                cb_init_launch<DIM, TYv, T, 0>(d, mask, v, x1, r, d0, x1, st);
            }
            // d1 holds d_1: iterations j >= 2 read D[(j - 1) & 1] = d1 first
            if (mass_sep == 0)
                cb_iterations3d<TYv, T, 0>(d, 2, mass_iters, d0, d1, r, x1, nullptr, nullptr, nullptr, mask, st);
            // steps 2 and 3 in three-term form on the 64 x 8 x mbz bricks (shorter halos than the 64 x 4
            // tiles): the start writes b (into r), and x_1 = s b only when it is the result (one iteration)
            {
                ProbeScope ps(d, KID_CHEB, st, (double)d.NT * (diff_iters == 1 ? 4.0 : 3.0) * sizeof(cx<T>), mask,
                              true);
                brick_depth(d, [&](auto bz) {
                    ps.launch(k_cb_init3d<decltype(bz)::value, kMassBY, T, 1>, dim3(d.nmtiles), dim3(kMassThreads),
                              d.sys, d.mtiles, mask, v, (const cx<T>*)x1, r, (cx<T>*)nullptr,
                              diff_iters == 1 ? x2 : (cx<T>*)nullptr, d.NT);
                });
            }
            cx_iterations3d<TYv, T>(d, diff_iters, d0, d1, r, x2, nullptr, nullptr, nullptr, mask, st);
            {
                ProbeScope ps(d, KID_CHEB, st, (double)d.NT * (diff_iters == 1 ? 3.0 : 2.0) * sizeof(cx<T>), mask,
                              true);
                brick_depth(d, [&](auto bz) {
                    ps.launch(k_cb_init3d<decltype(bz)::value, kMassBY, T, 2>, dim3(d.nmtiles), dim3(kMassThreads),
                              d.sys, d.mtiles, mask, v, (const cx<T>*)x2, r, (cx<T>*)nullptr,
                              diff_iters == 1 ? z + d.NT : (cx<T>*)nullptr, d.NT);
                });
            }
            // steps 3 and 4: the last iteration also forms z_zeta
            cx_iterations3d<TYv, T>(d, diff_iters, d0, d1, r, z + d.NT, x1, x2, z, mask, st);
            if (diff_iters < 2) {
                ProbeScope ps(d, KID_PC_FINAL, st);
                hipLaunchKernelGGL((k_pc_final<DIM, TYv, T>), TILE_GRID, d.sys, d.tiles, mask, x1, x2, z, d.NT);
            }
            return;
        }
        if (mass_sep > 0) {
            launch_mass_sep<T>(d, mass_sep, v, x1, mask, st);
        } else {
            {
                ProbeScope ps(d, KID_CHEB, st, (double)d.NT * 4.0 * sizeof(cx<T>), mask);
                cb_init_launch<DIM, TYv, T, 0>(d, mask, v, x1, r, d0, x1, st);
            }
            cb_iterations<DIM, TYv, T, 0>(d, mass_iters, d0, d1, r, x1, mask, st);
        }
        {
            ProbeScope ps(d, KID_CHEB, st, (double)d.NT * 5.0 * sizeof(cx<T>), mask);
            cb_init_launch<DIM, TYv, T, 1>(d, mask, v, x1, r, d0, x2, st);
        }
        cb_iterations<DIM, TYv, T, 1>(d, diff_iters, d0, d1, r, x2, mask, st);
        {
            ProbeScope ps(d, KID_CHEB, st, (double)d.NT * 4.0 * sizeof(cx<T>), mask);
            cb_init_launch<DIM, TYv, T, 2>(d, mask, v, x2, r, d0, z + d.NT, st);
        }
        cb_iterations<DIM, TYv, T, 1>(d, diff_iters, d0, d1, r, z + d.NT, mask, st);
        ProbeScope ps(d, KID_PC_FINAL, st);
        hipLaunchKernelGGL((k_pc_final<DIM, TYv, T>), TILE_GRID, d.sys, d.tiles, mask, x1, x2, z, d.NT);
    });
}
template void launch_precond_cheb_unfused<double>(const Dev&, const zd*, zd*, zd*, zd*, zd*, zd*, zd*, int, int, int,
                                                  const int*, hipStream_t);
template void launch_precond_cheb_unfused<float>(const Dev&, const zf*, zf*, zf*, zf*, zf*, zf*, zf*, int, int, int,
                                                 const int*, hipStream_t);

int brick_occupancy(int bz, bool single) {
    const void* f =
        single ? (bz == kBrickZDeep ? (const void*)&k_cx_iter3d<kBrickZDeep, kMassBY, float, false, false, false>
                                    : (const void*)&k_cx_iter3d<kBrickZShallow, kMassBY, float, false, false, false>)
               : (bz == kBrickZDeep ? (const void*)&k_cx_iter3d<kBrickZDeep, kMassBY, double, false, false, false>
                                    : (const void*)&k_cx_iter3d<kBrickZShallow, kMassBY, double, false, false, false>);
    int n = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, f, kMassThreads, 0) != hipSuccess) {
        (void)hipGetLastError();
        return 0;
    }
    return n;
}

template <typename T>
void launch_precond_mg(const Dev& d, const MgLevels& mg, const cx<T>* v, cx<T>* z, cx<T>* x1, cx<T>* x2, cx<T>* r,
                       cx<T>* d0, cx<T>* d1, cx<T>* b, int mass_iters, int mass_sep, const int* mask,
                       hipStream_t st) {
    dispatch(d, [&](auto D, auto TY) {
        constexpr int DIM = D(), TYv = TY();
        // step 1: beta1' ~ M^{-1} beta1 by the separable inverse or by Chebyshev iterations (as the Chebyshev
        // inner solver)
        if (mass_sep > 0) {
            launch_mass_sep<T>(d, mass_sep, v, x1, mask, st);
        } else {
            {
                ProbeScope ps(d, KID_CHEB, st, (double)d.NT * 4.0 * sizeof(cx<T>), mask);
                cb_init_launch<DIM, TYv, T, 0>(d, mask, v, x1, r, d0, x1, st);
            }
            cb_iterations<DIM, TYv, T, 0>(d, mass_iters, d0, d1, r, x1, mask, st);
        }
        // step 2: b = beta2 - kappa G beta1' (the stage-1 start writes it to its residual argument), one V-cycle
        {
            ProbeScope ps(d, KID_CHEB, st, (double)d.NT * 5.0 * sizeof(cx<T>), mask);
            cb_init_launch<DIM, TYv, T, 1>(d, mask, v, x1, b, d0, d1, st);
        }
        launch_mg_vcycle<T>(d, mg, b, x2, r, d0, d1, mask, st);
        // step 3: b = M beta2', one V-cycle into the eta part of z
        {
            ProbeScope ps(d, KID_CHEB, st, (double)d.NT * 4.0 * sizeof(cx<T>), mask);
            cb_init_launch<DIM, TYv, T, 2>(d, mask, v, x2, b, d0, d1, st);
        }
        launch_mg_vcycle<T>(d, mg, b, z + d.NT, r, d0, d1, mask, st);
        // step 4
        ProbeScope ps(d, KID_PC_FINAL, st);
        hipLaunchKernelGGL((k_pc_final<DIM, TYv, T>), TILE_GRID, d.sys, d.tiles, mask, x1, x2, z, d.NT);
    });
}
template void launch_precond_mg<double>(const Dev&, const MgLevels&, const zd*, zd*, zd*, zd*, zd*, zd*, zd*, zd*, int,
                                        int, const int*, hipStream_t);
template void launch_precond_mg<float>(const Dev&, const MgLevels&, const zf*, zf*, zf*, zf*, zf*, zf*, zf*, zf*, int,
                                       int, const int*, hipStream_t);

void launch_mass_solve(const Dev& d, const zd* eta, zd* zeta, zd* r, zd* p0, zd* p1, zd* q, double* part, int iters,
                       hipStream_t st) {
    // zeta = M^{-1} G eta by Chebyshev-Jacobi iterations with the exact bounds of D^{-1} M
    // ([1/2, 3/2]^dim): the error contracts by (sqrt(3^dim) - 1)/(sqrt(3^dim) + 1) per iteration.
    (void)q;
    (void)part;
    dispatch(d, [&](auto D, auto TY) {
        constexpr int DIM = D(), TYv = TY();
        cb_init_launch<DIM, TYv, double, 3>(d, nullptr, nullptr, eta, r, p0, zeta, st);
        cb_iterations<DIM, TYv, double, 0>(d, iters, p0, p1, r, zeta, nullptr, st);
    });
}

void launch_reduce(const Dev& d, const double* part, int slot0, int nvals, bool chunk_ranges, double* out, int ld,
                   const int* mask, hipStream_t st) {
    ProbeScope ps(d, KID_REDUCE, st);
    const long long P = chunk_ranges ? d.nchunks : d.ntiles;
    int gy = (nvals + 3) / 4;
    if (gy > 16) gy = 16;
    hipLaunchKernelGGL(k_reduce, dim3(d.S, gy), dim3(kBlock), 0, st, d.sys, mask, part, P, slot0, nvals, chunk_ranges,
                       out, ld);
}

template <typename VT>
void launch_gs(const Dev& d, const Krylov& kr, int k, const double* part1, const VT* V, long long vstride,
               const VT* w, double* part2, hipStream_t st) {
    // the second pass, where it runs, reads w and nv basis vectors (all stored in the basis precision)
    ProbeScope ps(d, KID_GS, st, 2.0 * d.NT * (k + 2) * sizeof(VT), kr.reorth);
    const int per = d.S >= kGsGrid ? 1 : (kGsGrid + d.S - 1) / d.S;
    const dim3 grid(d.S * per);
    const int nv = k + 1;
    auto go = [&](auto nvc) {
        hipLaunchKernelGGL((k_gs<decltype(nvc)::value, VT>), grid, dim3(kBlock), 0, st, d.sys, d.chunks, kr, d.S, k,
                           part1, (long long)d.ntiles, V, vstride, w, part2, d.nchunks, d.NT);
    };
    if (nv <= 4) go(std::integral_constant<int, 4>{});
    else if (nv <= 8) go(std::integral_constant<int, 8>{});
    else if (nv <= 16) go(std::integral_constant<int, 16>{});
    else go(std::integral_constant<int, 32>{});
}
template void launch_gs<zd>(const Dev&, const Krylov&, int, const double*, const zd*, long long, const zd*, double*,
                            hipStream_t);
template void launch_gs<zf>(const Dev&, const Krylov&, int, const double*, const zf*, long long, const zf*, double*,
                            hipStream_t);


template <typename VT>
void launch_proj_final(const Dev& d, const VT* V, long long vstride, int nv, const VT* w, const double* hcoef,
                       const double* hinv, int hstride, VT* out, const int* mask, hipStream_t st) {
    ProbeScope ps(d, KID_PROJ_FINAL, st, 2.0 * d.NT * (nv + 2) * sizeof(VT), mask);
    hipLaunchKernelGGL(k_proj_final<VT>, CHUNK_GRID, d.sys, d.chunks, mask, V, vstride, nv, w, hcoef, hstride, hinv, out,
                       d.NT);
}
template <typename VT>
void launch_scale(const Dev& d, const VT* r, const double* inv_beta, VT* v0, const int* mask, hipStream_t st) {
    hipLaunchKernelGGL(k_scale<VT>, CHUNK_GRID, d.sys, d.chunks, mask, r, inv_beta, v0, d.NT);
}
template void launch_proj_final<zd>(const Dev&, const zd*, long long, int, const zd*, const double*, const double*,
                                    int, zd*, const int*, hipStream_t);
template void launch_proj_final<zf>(const Dev&, const zf*, long long, int, const zf*, const double*, const double*,
                                    int, zf*, const int*, hipStream_t);
template void launch_scale<zd>(const Dev&, const zd*, const double*, zd*, const int*, hipStream_t);
template void launch_scale<zf>(const Dev&, const zf*, const double*, zf*, const int*, hipStream_t);
template <typename T>
void launch_xupdate(const Dev& d, const cx<T>* Z, long long zstride, const int* kcount, const double* y, int ldy,
                    zd* X, const int* mask, hipStream_t st) {
    ProbeScope ps(d, KID_XUPDATE, st);
    hipLaunchKernelGGL((k_xupdate<T>), CHUNK_GRID, d.sys, d.chunks, mask, Z, zstride, kcount, y, ldy, X, d.NT);
}
template void launch_xupdate<double>(const Dev&, const zd*, long long, const int*, const double*, int, zd*,
                                     const int*, hipStream_t);
template void launch_xupdate<float>(const Dev&, const zf*, long long, const int*, const double*, int, zd*,
                                    const int*, hipStream_t);

void launch_cycle_start(const Dev& d, const Krylov& kr, const double* part, bool first, int* pub, hipStream_t st) {
    ProbeScope ps(d, KID_SMALL, st);
    hipLaunchKernelGGL(k_cycle_start, dim3(d.S), dim3(kBlock), 0, st, d.sys, kr, d.S, first ? 1 : 0, part,
                       (long long)d.ntiles, pub);
}
void launch_solve_y(const Dev& d, const Krylov& kr, hipStream_t st) {
    ProbeScope ps(d, KID_SMALL, st);
    hipLaunchKernelGGL(k_solve_y, dim3((d.S + 63) / 64), dim3(64), 0, st, kr, d.S);
}

void launch_energy_parts(const Dev& d, const zd* eta, const zd* zeta, double* part, hipStream_t st) {
    dispatch(d, [&](auto D, auto TY) {
        hipLaunchKernelGGL((k_energy<D(), TY()>), TILE_GRID, d.sys, d.tiles, d.terms, eta, zeta, part, d.ntiles);
    });
}
void launch_energy_grad(const Dev& d, const zd* eta, const zd* zeta, double* const* grad_tab, double* part,
                        hipStream_t st) {
    dispatch(d, [&](auto D, auto TY) {
        hipLaunchKernelGGL((k_energy_grad<D(), TY()>), TILE_GRID, d.sys, d.tiles, d.terms, eta, zeta, grad_tab, part,
                           d.ntiles);
    });
}
void launch_rotation(const Dev& d, const zd* eta, double* const* omega_tab, double* const* h_tab, const RefineArgs& ra,
                     hipStream_t st) {
    dispatch(d, [&](auto D, auto TY) {
        hipLaunchKernelGGL((k_rotation<D(), TY()>), TILE_GRID, d.sys, d.tiles, d.terms, eta, omega_tab, h_tab, ra);
    });
}
void launch_adjoint_rhs(const Dev& d, double* const* lam_tab, zd* B, hipStream_t st) {
    dispatch(d, [&](auto D, auto TY) {
        hipLaunchKernelGGL((k_adjoint_rhs<D(), TY()>), TILE_GRID, d.sys, d.tiles, lam_tab, B, d.NT);
    });
}
void launch_adjoint_out(const Dev& d, const zd* Y, const zd* eta_prev, double* const* eta_new_tab,
                        double* const* lam_out_tab, double* part, hipStream_t st) {
    dispatch(d, [&](auto D, auto TY) {
        hipLaunchKernelGGL((k_adjoint_out<D(), TY()>), TILE_GRID, d.sys, d.tiles, d.terms, Y, eta_prev, eta_new_tab,
                           lam_out_tab, part, d.ntiles, d.NT);
    });
}

}  // namespace apfc
