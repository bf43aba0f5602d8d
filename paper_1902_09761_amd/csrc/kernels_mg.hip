// Geometric multigrid V-cycle for the diffusion operator L = M/sqrt(dt) + sqrt(kappa) K of the block
// preconditioner (Eq. (12)), the multigrid variant of its inner solves (Sec. III), on the structured mesh:
// levels of twice the mesh size, coarse operators by rediscretisation (the same stencil with the
// level's h, equal to the Galerkin product for the Q1 interpolation), symmetric Chebyshev-Jacobi
// smoothing (the level's Sys::cb[1] table: the upper part of the spectrum of D^{-1} L), restriction by
// the transpose of the Q1 interpolation, and a coarsest level solved in LDS by Chebyshev iterations over
// its whole spectrum.  One cycle from a zero initial guess:
//     x = S(b);  r = b - L x;  x += P V(P^T r);  r = b - L x;  x += S(r).
#include "kernels_common.h"

namespace apfc {

// (L u) at the node of n, u in the level's half vector
template <int DIM, typename T>
__device__ __forceinline__ cx<T> apply_L(const Sys& s, const Nbr<DIM>& n, const cx<T>* u) {
    cx<T> Mu, Ku, Tu;
    stencil<DIM, true, false, T>([&](int a, int b, int c) { return ld<T>(u, s.off + nb_index<DIM>(n, a, b, c)); },
                                 T(s.h), T(0), T(0), T(0), Mu, Ku, Tu);
    return T(s.isq_dt) * Mu + T(s.sq_kap) * Ku;
}

// Start of a smoothing pass.  ADD = false (from a zero guess): r = b, d = c0 b, x = d.
// ADD = true (a correction from the residual r): d = c0 r, x += d.
template <int DIM, int TY, typename T, bool ADD>
__global__ __launch_bounds__(kBlock) void k_mg_start(const Sys* sys, const Tile* tiles, const int* mask, const cx<T>* b,
                                                    cx<T>* r, cx<T>* d, cx<T>* xv) {
    TILE_PROLOGUE();
    const T c0 = T(sys[tile.sys].cb[1][0][0]);
    FOR_ROWS(TY) {
        const long long i = s.off + ((long long)pz * s.ny + y) * s.nx + x;
        if constexpr (ADD) {
            const cx<T> dv = c0 * ld<T>(r, i);
            d[i] = dv;
            xv[i] = ld<T>(xv, i) + dv;
        } else {
            const cx<T> bv = ld<T>(b, i);
            const cx<T> dv = c0 * bv;
            r[i] = bv;
            d[i] = dv;
            xv[i] = dv;
        }
    }
}

// Chebyshev iteration j >= 1 on L: r -= L d_{j-1}; d_j = c1 d_{j-1} + c2 r; x += d_j (LAST: r and d_j are
// not stored)
template <int DIM, int TY, typename T, bool LAST>
__global__ __launch_bounds__(kBlock) void k_mg_iter(const Sys* sys, const Tile* tiles, const int* mask, int j,
                                                   const cx<T>* din, cx<T>* dout, cx<T>* r, cx<T>* xv) {
    TILE_PROLOGUE();
    const T c1 = T(sys[tile.sys].cb[1][j][0]), c2 = T(sys[tile.sys].cb[1][j][1]);
    FOR_ROWS(TY) {
        Nbr<DIM> n;
        make_nbr<DIM>(s, x, y, pz, n);
        const long long i = s.off + nb_index<DIM>(n, 1, 1, 1);
        const cx<T> rv = ld<T>(r, i) - apply_L<DIM, T>(s, n, din);
        const cx<T> dv = c1 * ld<T>(din, i) + c2 * rv;
        xv[i] = ld<T>(xv, i) + dv;
        if constexpr (!LAST) {
            r[i] = rv;
            dout[i] = dv;
        }
    }
}

// r = b - L x
template <int DIM, int TY, typename T>
__global__ __launch_bounds__(kBlock) void k_mg_residual(const Sys* sys, const Tile* tiles, const int* mask,
                                                       const cx<T>* b, const cx<T>* xv, cx<T>* r) {
    TILE_PROLOGUE();
    FOR_ROWS(TY) {
        Nbr<DIM> n;
        make_nbr<DIM>(s, x, y, pz, n);
        const long long i = s.off + nb_index<DIM>(n, 1, 1, 1);
        r[i] = ld<T>(b, i) - apply_L<DIM, T>(s, n, xv);
    }
}

// Restriction b_c = P^T r_f on the coarse level's tiles: coarse node I gathers the fine nodes 2I + a,
// a in {-1, 0, 1}^dim (periodic), with weight prod_d (a_d == 0 ? 1 : 1/2).  fsys: the fine level's table
// (the same system index).
template <int DIM, int TY, typename T>
__global__ __launch_bounds__(kBlock) void k_mg_restrict(const Sys* sys, const Tile* tiles, const int* mask,
                                                       const Sys* fsys, const cx<T>* rf, cx<T>* bc) {
    TILE_PROLOGUE();
    const Sys f = fsys[tile.sys];
    FOR_ROWS(TY) {
        const int fx = 2 * x, fy = 2 * y, fz = 2 * pz;
        const int xs[3] = {fx == 0 ? f.nx - 1 : fx - 1, fx, fx + 1 == f.nx ? 0 : fx + 1};
        const int ys[3] = {fy == 0 ? f.ny - 1 : fy - 1, fy, fy + 1 == f.ny ? 0 : fy + 1};
        const int zs[3] = {DIM == 3 ? (fz == 0 ? f.nz - 1 : fz - 1) : 0, fz, DIM == 3 ? (fz + 1 == f.nz ? 0 : fz + 1) : 0};
        const T w[3] = {T(0.5), T(1), T(0.5)};
        cx<T> acc{T(0), T(0)};
#pragma unroll
        for (int c = (DIM == 3 ? 0 : 1); c < (DIM == 3 ? 3 : 2); ++c)
#pragma unroll
            for (int bb = 0; bb < 3; ++bb)
#pragma unroll
                for (int a = 0; a < 3; ++a) {
                    const T wt = w[a] * w[bb] * (DIM == 3 ? w[c] : T(1));
                    const long long fi = f.off + ((long long)zs[c] * f.ny + ys[bb]) * f.nx + xs[a];
                    acc = acc + wt * ld<T>(rf, fi);
                }
        bc[s.off + ((long long)pz * s.ny + y) * s.nx + x] = acc;
    }
}

// Prolongation x_f += P x_c on the fine level's tiles: per direction an even fine index 2i takes coarse
// node i, an odd one 2i + 1 the mean of coarse nodes i and i + 1 (periodic); tensor product.
template <int DIM, int TY, typename T>
__global__ __launch_bounds__(kBlock) void k_mg_prolong(const Sys* sys, const Tile* tiles, const int* mask,
                                                      const Sys* csys, const cx<T>* xc, cx<T>* xf) {
    TILE_PROLOGUE();
    const Sys c = csys[tile.sys];
    FOR_ROWS(TY) {
        int ix[2], iy[2], iz[2];
        T wx[2], wy[2], wz[2];
        auto par = [](int f, int nc, int (&i)[2], T (&w)[2]) {
            i[0] = f >> 1;
            if (f & 1) {
                i[1] = i[0] + 1 == nc ? 0 : i[0] + 1;
                w[0] = w[1] = T(0.5);
            } else {
                i[1] = i[0];
                w[0] = T(1);
                w[1] = T(0);
            }
        };
        par(x, c.nx, ix, wx);
        par(y, c.ny, iy, wy);
        if constexpr (DIM == 3) par(pz, c.nz, iz, wz);
        else { iz[0] = iz[1] = 0; wz[0] = T(1); wz[1] = T(0); }
        cx<T> acc{T(0), T(0)};
#pragma unroll
        for (int cz = 0; cz < 2; ++cz)
#pragma unroll
            for (int cy = 0; cy < 2; ++cy)
#pragma unroll
                for (int cxi = 0; cxi < 2; ++cxi) {
                    const T wt = wx[cxi] * wy[cy] * wz[cz];
                    if (wt != T(0))
                        acc = acc + wt * ld<T>(xc, c.off + ((long long)iz[cz] * c.ny + iy[cy]) * c.nx + ix[cxi]);
                }
        const long long i = s.off + ((long long)pz * s.ny + y) * s.nx + x;
        xf[i] = ld<T>(xf, i) + acc;
    }
}

// Coarsest level: x = Chebyshev^its(b) from zero over the whole spectrum (the level's cb[1] table), one
// workgroup per system with the level's correction d in LDS (at most kMgCoarseMax nodes), r and x of the
// thread's nodes in registers.
constexpr int kMgThreads = 1024;
constexpr int kMgPerThread = kMgCoarseMax / kMgThreads;

template <int DIM, typename T>
__global__ __launch_bounds__(kMgThreads) void k_mg_coarse(const Sys* sys, const int* mask, int its, const cx<T>* b,
                                                        cx<T>* xout) {
    __shared__ cx<T> dl[kMgCoarseMax];
    const int si = blockIdx.x;
    if (mask && !mask[si]) return;
    const Sys s = sys[si];
    const int N = (int)s.N;
    const double(*cb)[2] = sys[si].cb[1];
    const T cM = T(s.isq_dt), cK = T(s.sq_kap);
    cx<T> r[kMgPerThread], xv[kMgPerThread], dv[kMgPerThread];
    const T c0 = T(cb[0][0]);
#pragma unroll
    for (int q = 0; q < kMgPerThread; ++q) {
        const int i = (int)threadIdx.x + q * kMgThreads;
        if (i < N) {
            r[q] = ld<T>(b, s.off + i);
            dv[q] = c0 * r[q];
            xv[q] = dv[q];
        }
    }
    for (int k = 1; k < its; ++k) {
        __syncthreads();
#pragma unroll
        for (int q = 0; q < kMgPerThread; ++q) {
            const int i = (int)threadIdx.x + q * kMgThreads;
            if (i < N) dl[i] = dv[q];
        }
        __syncthreads();
        const T c1 = T(cb[k][0]), c2 = T(cb[k][1]);
#pragma unroll
        for (int q = 0; q < kMgPerThread; ++q) {
            const int i = (int)threadIdx.x + q * kMgThreads;
            if (i >= N) continue;
            const int ix = i % s.nx, iy = (i / s.nx) % s.ny, iz = DIM == 3 ? i / (s.nx * s.ny) : 0;
            const int xs[3] = {ix == 0 ? s.nx - 1 : ix - 1, ix, ix + 1 == s.nx ? 0 : ix + 1};
            const int ys[3] = {iy == 0 ? s.ny - 1 : iy - 1, iy, iy + 1 == s.ny ? 0 : iy + 1};
            const int zs[3] = {DIM == 3 ? (iz == 0 ? s.nz - 1 : iz - 1) : 0, iz, DIM == 3 ? (iz + 1 == s.nz ? 0 : iz + 1) : 0};
            cx<T> Mu, Ku, Tu;
            stencil<DIM, true, false, T>([&](int a, int bb, int c) { return dl[(zs[c] * s.ny + ys[bb]) * s.nx + xs[a]]; },
                                         T(s.h), T(0), T(0), T(0), Mu, Ku, Tu);
            r[q] = r[q] - (cM * Mu + cK * Ku);
            dv[q] = c1 * dv[q] + c2 * r[q];
            xv[q] = xv[q] + dv[q];
        }
    }
#pragma unroll
    for (int q = 0; q < kMgPerThread; ++q) {
        const int i = (int)threadIdx.x + q * kMgThreads;
        if (i < N) xout[s.off + i] = xv[q];
    }
}

// ------------------------------------------------------------------------------------------
// launchers
// ------------------------------------------------------------------------------------------
// smoothing on one level: from zero (ADD = false, b given) or as a correction from the residual r
// (ADD = true); nu Chebyshev iterations in all
template <int DIM, int TY, typename T, bool ADD>
static void mg_smooth(const Dev& d, int nu, const cx<T>* b, cx<T>* r, cx<T>* d0, cx<T>* d1, cx<T>* x, const int* mask,
                      hipStream_t st) {
    {
        // reads b or r (and x when ADD), writes r or d, d and x
        ProbeScope ps(d, KID_MG, st, (double)d.NT * sizeof(cx<T>) * (ADD ? 4.0 : 4.0), mask);
        hipLaunchKernelGGL((k_mg_start<DIM, TY, T, ADD>), TILE_GRID, d.sys, d.tiles, mask, b, r, d0, x);
    }
    cx<T>* D[2] = {d0, d1};
    for (int j = 1; j < nu; ++j) {
        const bool last = j == nu - 1;
        ProbeScope ps(d, KID_MG, st, (double)d.NT * sizeof(cx<T>) * (last ? 4.0 : 6.0), mask);
        if (last)
            hipLaunchKernelGGL((k_mg_iter<DIM, TY, T, true>), TILE_GRID, d.sys, d.tiles, mask, j, D[(j - 1) & 1],
                               D[j & 1], r, x);
        else
            hipLaunchKernelGGL((k_mg_iter<DIM, TY, T, false>), TILE_GRID, d.sys, d.tiles, mask, j, D[(j - 1) & 1],
                               D[j & 1], r, x);
    }
}

template <typename T>
void launch_mg_vcycle(const Dev& fine, const MgLevels& mg, const cx<T>* b, cx<T>* x, cx<T>* r, cx<T>* d0, cx<T>* d1,
                      const int* mask, hipStream_t st) {
    // level l: 0 = the fine level (the caller's buffers and tiles), 1..mg.n the coarser ones
    const int L = mg.n + 1;
    auto dev = [&](int l) -> const Dev& { return l == 0 ? fine : mg.lev[l - 1]; };
    auto B = [&](int l) { return l == 0 ? const_cast<cx<T>*>(b) : (cx<T>*)mg.b[l - 1]; };
    auto X = [&](int l) { return l == 0 ? x : (cx<T>*)mg.x[l - 1]; };
    auto R = [&](int l) { return l == 0 ? r : (cx<T>*)mg.r[l - 1]; };
    auto D0 = [&](int l) { return l == 0 ? d0 : (cx<T>*)mg.d0[l - 1]; };
    auto D1 = [&](int l) { return l == 0 ? d1 : (cx<T>*)mg.d1[l - 1]; };
    // down: smooth, residual, restrict
    for (int l = 0; l + 1 < L; ++l) {
        const Dev& d = dev(l);
        const Dev& dc = dev(l + 1);
        dispatch(d, [&](auto Dc, auto TYc) {
            constexpr int DIM = Dc(), TY = TYc();
            mg_smooth<DIM, TY, T, false>(d, mg.nu, B(l), R(l), D0(l), D1(l), X(l), mask, st);
            ProbeScope ps(d, KID_MG, st, (double)d.NT * sizeof(cx<T>) * 3.0, mask);
            hipLaunchKernelGGL((k_mg_residual<DIM, TY, T>), dim3(d.ntiles), dim3(kBlock), 0, st, d.sys, d.tiles, mask,
                               B(l), X(l), R(l));
        });
        dispatch(dc, [&](auto Dc, auto TYc) {
            constexpr int DIM = Dc(), TY = TYc();
            ProbeScope ps(dc, KID_MG, st, (double)dc.NT * sizeof(cx<T>) * (DIM == 3 ? 9.0 : 5.0), mask);
            hipLaunchKernelGGL((k_mg_restrict<DIM, TY, T>), dim3(dc.ntiles), dim3(kBlock), 0, st, dc.sys, dc.tiles,
                               mask, d.sys, R(l), B(l + 1));
        });
    }
    // coarsest level
    {
        const Dev& d = dev(L - 1);
        ProbeScope ps(d, KID_MG, st, (double)d.NT * sizeof(cx<T>) * 2.0, mask);
        if (d.dim == 3)
            hipLaunchKernelGGL((k_mg_coarse<3, T>), dim3(d.S), dim3(kMgThreads), 0, st, d.sys, mask, mg.coarse_its,
                               B(L - 1), X(L - 1));
        else
            hipLaunchKernelGGL((k_mg_coarse<2, T>), dim3(d.S), dim3(kMgThreads), 0, st, d.sys, mask, mg.coarse_its,
                               B(L - 1), X(L - 1));
    }
    // up: prolong, residual, smooth the correction
    for (int l = L - 2; l >= 0; --l) {
        const Dev& d = dev(l);
        const Dev& dc = dev(l + 1);
        dispatch(d, [&](auto Dc, auto TYc) {
            constexpr int DIM = Dc(), TY = TYc();
            {
                ProbeScope ps(d, KID_MG, st, (double)d.NT * sizeof(cx<T>) * (2.0 + 1.0 / (1 << DIM)), mask);
                hipLaunchKernelGGL((k_mg_prolong<DIM, TY, T>), dim3(d.ntiles), dim3(kBlock), 0, st, d.sys, d.tiles,
                                   mask, dc.sys, X(l + 1), X(l));
            }
            {
                ProbeScope ps(d, KID_MG, st, (double)d.NT * sizeof(cx<T>) * 3.0, mask);
                hipLaunchKernelGGL((k_mg_residual<DIM, TY, T>), dim3(d.ntiles), dim3(kBlock), 0, st, d.sys, d.tiles,
                                   mask, B(l), X(l), R(l));
            }
            mg_smooth<DIM, TY, T, true>(d, mg.nu, nullptr, R(l), D0(l), D1(l), X(l), mask, st);
        });
    }
}
template void launch_mg_vcycle<double>(const Dev&, const MgLevels&, const zd*, zd*, zd*, zd*, zd*, const int*,
                                       hipStream_t);
template void launch_mg_vcycle<float>(const Dev&, const MgLevels&, const zf*, zf*, zf*, zf*, zf*, const int*,
                                      hipStream_t);

}  // namespace apfc
