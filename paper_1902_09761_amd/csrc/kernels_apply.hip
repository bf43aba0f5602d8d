// HIP kernels of the block operator A_j (Eq. (11)) for gfx950: the plain apply, the 2D column march and
// the 3D plane march with the first Gram-Schmidt pass fused (k_apply_dot2d/3d), and the true residual
// (k_residual2d/3d), with their launchers.
#include "kernels_common.h"

namespace apfc {

// ------------------------------------------------------------------------------------------
// block operator A_j (Eq. (11)): y1 = M zeta - G eta,  y2 = kappa G zeta + M eta/dt + kappa w d eta
// ------------------------------------------------------------------------------------------
template <int DIM, typename S>
__device__ __forceinline__ void apply_A(const Sys& s, const Nbr<DIM>& n, const cx<S>* zz, const cx<S>* ze, double dn,
                                        zd& y1, zd& y2) {
    zd Mz, Kz, Tz, Me, Ke, Te;
    stencil<DIM, true, true, double>(
        [&](int a, int b, int c) { return ld<double>(zz, s.off + nb_index<DIM>(n, a, b, c)); }, s.h, s.kv[0],
        s.kv[1], s.kv[2], Mz, Kz, Tz);
    stencil<DIM, true, true, double>(
        [&](int a, int b, int c) { return ld<double>(ze, s.off + nb_index<DIM>(n, a, b, c)); }, s.h, s.kv[0],
        s.kv[1], s.kv[2], Me, Ke, Te);
    const zd ec = ld<double>(ze, s.off + nb_index<DIM>(n, 1, 1, 1));
    y1 = Mz - gop(Ke, Te);
    y2 = s.kappa * gop(Kz, Tz) + s.inv_dt * Me + (s.kappa * s.w * dn) * ec;
}

template <int DIM, int TY, typename T>
__global__ __launch_bounds__(kBlock) void k_apply(const Sys* sys, const Tile* tiles, const int* mask,
                                                 const cx<T>* Z, const double* dnode, zd* W, long long NT) {
    TILE_PROLOGUE();
    FOR_ROWS(TY) {
        Nbr<DIM> n;
        make_nbr<DIM>(s, x, y, pz, n);
        const long long il = nb_index<DIM>(n, 1, 1, 1);
        zd y1, y2;
        apply_A<DIM, T>(s, n, Z, Z + NT, dnode[s.doff + il], y1, y2);
        W[s.off + il] = y1;
        W[NT + s.off + il] = y2;
    }
}

// 2D column march: a thread walks rows y0-1 .. y0+RR of column x (periodic); the x pass (mass,
// stiffness, derivative sums over x-1, x, x+1) of every row is computed once and kept for the next
// two rows, so each input row is loaded once per field (3 loads instead of 9).  load(f, i) returns node i
// of the system's zeta (f = 0) or eta (f = 1) part of u; emit(il, y1, y2) receives A_j u at node
// il = (x, y) for y = y0 .. y0+RR-1 inside the mesh.  CHECK = false: the caller knows that every row and
// column of the march lies inside the mesh, so the march has no branch and the compiler can issue the
// loads of later rows while earlier rows are computed.
template <int RR, bool CHECK, typename LOAD, typename EMIT>
__device__ __forceinline__ void colmarch_A(const Sys& s, int x, int y0, const LOAD& load, const double* dnode,
                                           const EMIT& emit) {
    const int xc = x < s.nx ? x : s.nx - 1;                  // clamp for loads of ragged tiles
    const int xm = xc == 0 ? s.nx - 1 : xc - 1, xp = xc == s.nx - 1 ? 0 : xc + 1;
    const double h = s.h, m0 = h / 6.0, m1 = 4.0 * h / 6.0, ih = 1.0 / h;
    const double kx = s.kv[0], ky = s.kv[1];
    zd mz[3], kz[3], dz[3], me[3], ke[3], de[3], ce[3];
    // first row y0 - 1, periodic; y0 itself may lie past the mesh (rows of a tile taller than the mesh)
    int row = y0 == 0 ? s.ny - 1 : (y0 - 1) % s.ny;
#pragma unroll
    for (int a = 0; a < RR + 2; ++a, row = row + 1 == s.ny ? 0 : row + 1) {
        const long long rb = (long long)row * s.nx;
        {
            const zd l = load(0, rb + xm), c = load(0, rb + xc), r = load(0, rb + xp);
            mz[2] = m0 * (l + r) + m1 * c;
            kz[2] = ih * ((c + c) - (l + r));
            dz[2] = 0.5 * (r - l);
        }
        {
            const zd l = load(1, rb + xm), c = load(1, rb + xc), r = load(1, rb + xp);
            me[2] = m0 * (l + r) + m1 * c;
            ke[2] = ih * ((c + c) - (l + r));
            de[2] = 0.5 * (r - l);
            ce[2] = c;
        }
        if (a >= 2) {
            const int y = y0 + a - 2;
            if (!CHECK || (x < s.nx && y < s.ny)) {
                auto Msum = [&](const zd* u) { return m0 * (u[0] + u[2]) + m1 * u[1]; };
                const zd Mz = Msum(mz), Me = Msum(me);
                const zd Kz = Msum(kz) + ih * ((mz[1] + mz[1]) - (mz[0] + mz[2]));
                const zd Ke = Msum(ke) + ih * ((me[1] + me[1]) - (me[0] + me[2]));
                const zd Tz = 2.0 * (kx * Msum(dz) + ky * (0.5 * (mz[2] - mz[0])));
                const zd Te = 2.0 * (kx * Msum(de) + ky * (0.5 * (me[2] - me[0])));
                const long long il = (long long)y * s.nx + x;
                const zd y1 = Mz - gop(Ke, Te);
                const zd y2 = s.kappa * gop(Kz, Tz) + s.inv_dt * Me + (s.kappa * s.w * dnode[s.doff + il]) * ce[1];
                emit(il, y1, y2);
            }
        }
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            mz[j] = mz[j + 1]; kz[j] = kz[j + 1]; dz[j] = dz[j + 1];
            me[j] = me[j + 1]; ke[j] = ke[j + 1]; de[j] = de[j + 1]; ce[j] = ce[j + 1];
        }
    }
}

// W = A Z at every node and, fused, the first Gram-Schmidt pass: per-tile partials of V_i^H w
// (i < nv) and of |w|^2 (slots 2i, 2i+1 and 2 nv of part, stride ntiles).  2D: column-marching
// tiles (TY/4 rows per thread); 3D: k_apply_dot3d below.
// NV >= nv basis vectors; with NV <= 8 the launch uses NV = nv exactly, so the basis loads carry no test.
template <int TY, typename T, int NV>
__global__ __launch_bounds__(kBlock) void k_apply_dot2d(const Sys* sys, const Tile* tiles, const int* mask,
                                                       const cx<T>* __restrict__ Z, const double* __restrict__ dnode,
                                                       cx<T>* __restrict__ W, const cx<T>* __restrict__ V,
                                                       long long vstride, int nv, double* part, long long NT,
                                                       int ntiles) {
    constexpr int RR = TY / 4;
    __shared__ double lds[4 * (2 * NV + 1)];
    TILE_PROLOGUE();
    const int y0 = tile.y0 + ty * RR;
    double acc[2 * NV + 1];
#pragma unroll
    for (int i = 0; i < 2 * NV + 1; ++i) acc[i] = 0.0;
    const cx<T>* zz = Z + s.off;
    const cx<T>* ze = Z + NT + s.off;
    auto load = [&](int f, long long i) { return ld<double>(f == 0 ? zz : ze, i); };
    auto emit = [&](long long il, const zd& a1, const zd& a2) {
        // w is stored in the basis precision; the first pass takes the stored (rounded) w, so that the
        // projection of k_proj_final and the coefficients belong to the same vector
        const zd y1 = rounded<T>(a1), y2 = rounded<T>(a2);
        stv(W, s.off + il, y1);
        stv(W, NT + s.off + il, y2);
        acc[2 * NV] += abs2(y1) + abs2(y2);
#pragma unroll
        for (int l = 0; l < NV; ++l)
            if (NV <= 8 || l < nv) {
                const zd p = cdot(ld<double>(V, l * vstride + s.off + il), y1),
                         q = cdot(ld<double>(V, l * vstride + NT + s.off + il), y2);
                acc[2 * l] += p.x + q.x;
                acc[2 * l + 1] += p.y + q.y;
            }
    };
    if (tile.x0 + 64 <= s.nx && y0 + RR <= s.ny)
        colmarch_A<RR, false>(s, x, y0, load, dnode, emit);
    else
        colmarch_A<RR, true>(s, x, y0, load, dnode, emit);
    block_sum<2 * NV + 1>(acc, lds);
    if (threadIdx.x == 0) {
#pragma unroll
        for (int l = 0; l < NV; ++l)
            if (l < nv) {
                part[(2 * l) * (long long)ntiles + blockIdx.x] = acc[2 * l];
                part[(2 * l + 1) * (long long)ntiles + blockIdx.x] = acc[2 * l + 1];
            }
        part[(2 * nv) * (long long)ntiles + blockIdx.x] = acc[2 * NV];
    }
}

// R = B - A X and per-tile partials of |R|^2, |B|^2 (slots kRR, kBB), on column-marching tiles.
// R is stored in precision RT (the Krylov basis precision: only v_0 = r / |r| is formed from it); the
// norms come from the FP64 values.
template <int TY, typename RT>
__global__ __launch_bounds__(kBlock) void k_residual2d(const Sys* sys, const Tile* tiles, const int* mask,
                                                      const zd* __restrict__ X, const zd* __restrict__ B,
                                                      const double* __restrict__ dnode, RT* __restrict__ R,
                                                      double* part, long long NT, int ntiles) {
    constexpr int RR = TY / 4;
    __shared__ double lds[8];
    TILE_PROLOGUE();
    const int y0 = tile.y0 + ty * RR;
    double acc[2] = {0.0, 0.0};
    const zd* xz = X + s.off;
    const zd* xe = X + NT + s.off;
    auto load = [&](int f, long long i) { return (f == 0 ? xz : xe)[i]; };
    auto emit = [&](long long il, const zd& y1, const zd& y2) {
        const zd b1 = B[s.off + il], b2 = B[NT + s.off + il];
        const zd r1 = b1 - y1, r2 = b2 - y2;
        stv(R, s.off + il, r1);
        stv(R, NT + s.off + il, r2);
        acc[0] += abs2(r1) + abs2(r2);
        acc[1] += abs2(b1) + abs2(b2);
    };
    if (tile.x0 + 64 <= s.nx && y0 + RR <= s.ny)
        colmarch_A<RR, false>(s, x, y0, load, dnode, emit);
    else
        colmarch_A<RR, true>(s, x, y0, load, dnode, emit);
    block_sum<2>(acc, lds);
    if (threadIdx.x == 0) {
        part[kRR * (long long)ntiles + blockIdx.x] = acc[0];
        part[kBB * (long long)ntiles + blockIdx.x] = acc[1];
    }
}

// 3D versions of k_apply_dot2d and k_residual2d on z-marching bricks (64 x 4 x TY/4 nodes).
#define BRICK_PROLOGUE()                                                     \
    TILE_PROLOGUE();                                                         \
    const int y = tile.y0 + ty;                                              \
    const int xc = x < s.nx ? x : s.nx - 1, yc = y < s.ny ? y : s.ny - 1;    \
    const double m0 = s.h * (1.0 / 6.0), m1 = s.h * (4.0 / 6.0), ih = 1.0 / s.h;

template <int TY, typename T, int NV>
__global__ __launch_bounds__(kBlock) void k_apply_dot3d(const Sys* sys, const Tile* tiles, const int* mask,
                                                       const cx<T>* Z, const double* dnode, cx<T>* W, const cx<T>* V,
                                                       long long vstride, int nv, double* part, long long NT,
                                                       int ntiles) {
    __shared__ double lds[4 * (2 * NV + 1)];
    BRICK_PROLOGUE();
    const cx<T>* zz = Z + s.off;
    const cx<T>* ze = Z + NT + s.off;
    double acc[2 * NV + 1];
#pragma unroll
    for (int i = 0; i < 2 * NV + 1; ++i) acc[i] = 0.0;
    auto emit = [&](int z, const auto& P) {
        if (x >= s.nx || y >= s.ny || z >= s.nz) return;
        const long long il = ((long long)z * s.ny + y) * s.nx + x;
        zd a1, a2;
        apply_A_planes(s, P, m0, m1, ih, dnode[s.doff + il], a1, a2);
        const zd y1 = rounded<T>(a1), y2 = rounded<T>(a2);
        stv(W, s.off + il, y1);
        stv(W, NT + s.off + il, y2);
        acc[2 * NV] += abs2(y1) + abs2(y2);
#pragma unroll
        for (int l = 0; l < NV; ++l)
            if (NV <= 8 || l < nv) {
                const zd p = cdot(ld<double>(V, l * vstride + s.off + il), y1),
                     q = cdot(ld<double>(V, l * vstride + NT + s.off + il), y2);
                acc[2 * l] += p.x + q.x;
                acc[2 * l + 1] += p.y + q.y;
            }
    };
    // FP32 storage: the next plane's values are loaded while the current one is used (two waves per SIMD
    // either way); FP64 storage keeps the plain march, whose look-ahead would halve its waves
    if constexpr (sizeof(T) == 4)
        zmarch_prefetch<TY / 4, 2, true, true, double, T>(s, xc, yc, tile.z, m0, m1, ih,
                                                          [&](int f) { return f == 0 ? zz : ze; }, emit);
    else
        zmarch<TY / 4, 2, true, true, double>(
            s, xc, yc, tile.z, m0, m1, ih, [&](int f, long long i) { return ld<double>(f == 0 ? zz : ze, i); }, emit);
    block_sum<2 * NV + 1>(acc, lds);
    if (threadIdx.x == 0) {
#pragma unroll
        for (int l = 0; l < NV; ++l)
            if (l < nv) {
                part[(2 * l) * (long long)ntiles + blockIdx.x] = acc[2 * l];
                part[(2 * l + 1) * (long long)ntiles + blockIdx.x] = acc[2 * l + 1];
            }
        part[(2 * nv) * (long long)ntiles + blockIdx.x] = acc[2 * NV];
    }
}

template <int TY, typename RT>
__global__ __launch_bounds__(kBlock) void k_residual3d(const Sys* sys, const Tile* tiles, const int* mask, const zd* X,
                                                      const zd* B, const double* dnode, RT* R, double* part,
                                                      long long NT, int ntiles) {
    __shared__ double lds[8];
    BRICK_PROLOGUE();
    const zd* xz = X + s.off;
    const zd* xe = X + NT + s.off;
    double acc[2] = {0.0, 0.0};
    zmarch<TY / 4, 2, true, true, double>(
        s, xc, yc, tile.z, m0, m1, ih, [&](int f, long long i) { return (f == 0 ? xz : xe)[i]; },
        [&](int z, const auto& P) {
            if (x >= s.nx || y >= s.ny || z >= s.nz) return;
            const long long il = ((long long)z * s.ny + y) * s.nx + x;
            zd y1, y2;
            apply_A_planes(s, P, m0, m1, ih, dnode[s.doff + il], y1, y2);
            const zd b1 = B[s.off + il], b2 = B[NT + s.off + il];
            const zd r1 = b1 - y1, r2 = b2 - y2;
            stv(R, s.off + il, r1);
            stv(R, NT + s.off + il, r2);
            acc[0] += abs2(r1) + abs2(r2);
            acc[1] += abs2(b1) + abs2(b2);
        });
    block_sum<2>(acc, lds);
    if (threadIdx.x == 0) {
        part[kRR * (long long)ntiles + blockIdx.x] = acc[0];
        part[kBB * (long long)ntiles + blockIdx.x] = acc[1];
    }
}

template <typename RT>
void launch_residual(const Dev& d, const zd* X, const zd* B, const double* dnode, RT* R, double* part,
                     const int* mask, hipStream_t st) {
    ProbeScope ps(d, KID_RESIDUAL, st, (double)d.NT * (4.0 * sizeof(zd) + 2.0 * sizeof(RT) + 8.0 / d.J), mask);
    dispatch(d, [&](auto D, auto TY) {
        if constexpr (D() == 3)
            hipLaunchKernelGGL((k_residual3d<TY(), RT>), TILE_GRID, d.sys, d.tiles, mask, X, B, dnode, R, part, d.NT,
                               d.ntiles);
        else
            hipLaunchKernelGGL((k_residual2d<TY(), RT>), TILE_GRID, d.sys, d.tiles, mask, X, B, dnode, R, part, d.NT,
                               d.ntiles);
    });
}
template void launch_residual<zd>(const Dev&, const zd*, const zd*, const double*, zd*, double*, const int*,
                                  hipStream_t);
template void launch_residual<zf>(const Dev&, const zd*, const zd*, const double*, zf*, double*, const int*,
                                  hipStream_t);
template <typename T>
void launch_apply(const Dev& d, const cx<T>* Z, const double* dnode, zd* W, const int* mask, hipStream_t st) {
    // reads z (2 half vectors) and d (per instance), writes w (2 FP64 half vectors)
    ProbeScope ps(d, KID_APPLY, st, (double)d.NT * (2.0 * sizeof(cx<T>) + 2.0 * sizeof(zd) + 8.0 / d.J), mask);
    dispatch(d, [&](auto D, auto TY) {
        hipLaunchKernelGGL((k_apply<D(), TY(), T>), TILE_GRID, d.sys, d.tiles, mask, Z, dnode, W, d.NT);
    });
}
template void launch_apply<double>(const Dev&, const zd*, const double*, zd*, const int*, hipStream_t);
template void launch_apply<float>(const Dev&, const zf*, const double*, zd*, const int*, hipStream_t);

template <typename T>
void launch_apply_dot(const Dev& d, const cx<T>* Z, const double* dnode, cx<T>* W, const cx<T>* V, long long vstride,
                      int nv, double* part, const int* mask, hipStream_t st) {
    // reads z, d, nv basis vectors (stored like z); writes w (stored like z)
    ProbeScope ps(d, KID_APPLY, st, (double)d.NT * (2.0 * sizeof(cx<T>) * (2 + nv) + 8.0 / d.J), mask, true);
    dispatch(d, [&](auto D, auto TY) {
        auto go = [&](auto nvc) {
            if constexpr (D() == 2)
                ps.launch(k_apply_dot2d<TY(), T, decltype(nvc)::value>, dim3(d.ntiles), dim3(kBlock), d.sys, d.tiles,
                          mask, Z, dnode, W, V, vstride, nv, part, d.NT, d.ntiles);
            else
                ps.launch(k_apply_dot3d<TY(), T, decltype(nvc)::value>, dim3(d.ntiles), dim3(kBlock), d.sys, d.tiles,
                          mask, Z, dnode, W, V, vstride, nv, part, d.NT, d.ntiles);
        };
        switch (nv) {
            case 1: go(std::integral_constant<int, 1>{}); return;
            case 2: go(std::integral_constant<int, 2>{}); return;
            case 3: go(std::integral_constant<int, 3>{}); return;
            case 4: go(std::integral_constant<int, 4>{}); return;
            case 5: go(std::integral_constant<int, 5>{}); return;
            case 6: go(std::integral_constant<int, 6>{}); return;
            case 7: go(std::integral_constant<int, 7>{}); return;
            case 8: go(std::integral_constant<int, 8>{}); return;
            default: break;
        }
        if (nv <= 16) go(std::integral_constant<int, 16>{});
        else go(std::integral_constant<int, 32>{});
    });
}
template void launch_apply_dot<double>(const Dev&, const zd*, const double*, zd*, const zd*, long long, int, double*,
                                       const int*, hipStream_t);
template void launch_apply_dot<float>(const Dev&, const zf*, const double*, zf*, const zf*, long long, int, double*,
                                      const int*, hipStream_t);

}  // namespace apfc
