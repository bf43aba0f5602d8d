// Step 1 of the block preconditioner (Eq. (12), the mass solve M x1 = beta1) by a separable approximate
// inverse of the mass matrix, for gfx950, with its launcher.
#include "kernels_common.h"

namespace apfc {

// On the uniform periodic mesh the Q1 mass matrix is the Kronecker product of the 1D matrices
// (h/6) tridiag(1, 4, 1) of the directions, so its inverse is the Kronecker product of their inverses.
// The 1D inverse has the entries (sqrt(3)/h) rho^|k| with rho = sqrt(3) - 2, which fall by |rho| ~ 0.27
// per node; W keeps |k| <= R in each direction, so x1 = W beta1 is one 1D filter of 2R + 1 taps per
// direction (Sys::wsep holds (sqrt(3)/h) rho^k).  Taps that wrap onto the same node of a short periodic
// direction add up.
//
// A workgroup of 512 threads owns a brick of 64 x kMassBY nodes per plane and BZ planes (one plane in
// 2D).  For each plane, from R planes before the brick to R planes after it (periodic), it stages the
// plane's region of (64 + 2R) x (kMassBY + 2R) nodes in LDS (the next plane's loads in flight meanwhile),
// filters the region's rows in x into a second LDS array, filters that in y at the thread's node and keeps
// the last 2R + 1 such values of its column in registers for the z filter.  HBM traffic: beta1 read once
// (the halos come from L2) and x1 written once; about 4 (2D) and 7 (3D) multiply-adds per tap and node.
__device__ __forceinline__ int wrapm(int g, int n) {
    g %= n;
    return g < 0 ? g + n : g;
}

template <int DIM, int BZ, typename T, int R>
__global__ __launch_bounds__(kMassThreads) void k_mass_sep(const Sys* sys, const Tile* tiles, const int* mask,
                                                          const cx<T>* __restrict__ v, cx<T>* __restrict__ x1) {
    constexpr int PX = kTX + 2 * R, PY = kMassBY + 2 * R, PP = PX * PY;
    constexpr int NZ = DIM == 3 ? BZ + 2 * R : 1;   // planes marched
    static_assert(kMassThreads == kTX * kMassBY, "one thread per node of a brick plane");
    constexpr int NS = (PP + kMassThreads - 1) / kMassThreads;   // staged nodes per thread and plane
    __shared__ cx<T> A[PP];
    __shared__ cx<T> B[PY * kTX];
    const Tile tile = tiles[blockIdx.x];
    if (mask && !mask[tile.sys]) return;
    const Sys* sp = sys + tile.sys;
    const int nx = sp->nx, ny = sp->ny, nz = sp->nz;
    const long long off = sp->off, plane = (long long)nx * ny;
    T w[R + 1];
#pragma unroll
    for (int k = 0; k <= R; ++k) w[k] = T(sp->wsep[k]);
    const int t = (int)threadIdx.x, lx = t % kTX, ly = t / kTX;
    static_assert(NS <= 3, "at most three staged nodes per thread");
    // the thread's staged nodes t, t + 512, t + 1024 of a plane region (offsets inside the plane)
    auto goff = [&](int e) -> long long {
        const int gx = wrapm(tile.x0 - R + e % PX, nx), gy = wrapm(tile.y0 - R + e / PX, ny);
        return e < PP ? (long long)gy * nx + gx : 0;
    };
    const long long o0 = goff(t), o1 = NS > 1 ? goff(t + kMassThreads) : 0, o2 = NS > 2 ? goff(t + 2 * kMassThreads) : 0;
    const bool h1 = NS > 1 && t + kMassThreads < PP, h2 = NS > 2 && t + 2 * kMassThreads < PP;
    const cx<T> zero{T(0), T(0)};
    int zz = DIM == 3 ? wrapm(tile.z - R, nz) : 0;
    cx<T> a0 = zero, a1 = zero, a2 = zero;
    auto fetch = [&](long long base) {
        a0 = v[base + o0];
        if (h1) a1 = v[base + o1];
        if (h2) a2 = v[base + o2];
    };
    fetch(off + zz * plane);
    cx<T> Q[2 * R + 1];
#pragma unroll
    for (int i = 0; i < 2 * R + 1; ++i) Q[i] = zero;
    const int x = tile.x0 + lx, y = tile.y0 + ly;
#pragma unroll 1
    for (int p = 0; p < NZ; ++p) {
        __syncthreads();   // every read of A (x filter) and B (y filter) of the previous plane is done
        A[t] = a0;
        if (h1) A[t + kMassThreads] = a1;
        if (h2) A[t + 2 * kMassThreads] = a2;
        if (p + 1 < NZ) {
            zz = zz + 1 == nz ? 0 : zz + 1;
            fetch(off + zz * plane);
        }
        __syncthreads();
        // x filter of every region row at the 64 brick columns
        for (int e = t; e < PY * kTX; e += kMassThreads) {
            const cx<T>* row = A + (e / kTX) * PX + (e % kTX) + R;
            cx<T> acc = w[0] * row[0];
#pragma unroll
            for (int k = 1; k <= R; ++k) acc = acc + w[k] * (row[-k] + row[k]);
            B[e] = acc;
        }
        __syncthreads();
        // y filter at the thread's node
        const cx<T>* col = B + (ly + R) * kTX + lx;
        cx<T> u = w[0] * col[0];
#pragma unroll
        for (int k = 1; k <= R; ++k) u = u + w[k] * (col[-k * kTX] + col[k * kTX]);
        if constexpr (DIM == 2) {
            if (x < nx && y < ny) x1[off + (long long)y * nx + x] = u;
        } else {
            // Q[i] holds the filtered plane tile.z - 3R + p + i; the z filter is centred on Q[R]
#pragma unroll
            for (int i = 0; i < 2 * R; ++i) Q[i] = Q[i + 1];
            Q[2 * R] = u;
            const int z = tile.z + p - 2 * R;
            if (p >= 2 * R && x < nx && y < ny && z < nz) {
                cx<T> o = w[0] * Q[R];
#pragma unroll
                for (int k = 1; k <= R; ++k) o = o + w[k] * (Q[R - k] + Q[R + k]);
                x1[off + ((long long)z * ny + y) * nx + x] = o;
            }
        }
    }
}

template <typename T>
void launch_mass_sep(const Dev& d, int R, const cx<T>* v, cx<T>* x1, const int* mask, hipStream_t st) {
    ProbeScope ps(d, KID_MASS, st, (double)d.NT * 2.0 * sizeof(cx<T>), mask, true);
    auto go = [&](auto rc) {
        constexpr int RR = decltype(rc)::value;
        if (d.dim == 3)
            brick_depth(d, [&](auto bz) {
                ps.launch(k_mass_sep<3, decltype(bz)::value, T, RR>, dim3(d.nmtiles), dim3(kMassThreads), d.sys,
                          d.mtiles, mask, v, x1);
            });
        else
            ps.launch(k_mass_sep<2, 1, T, RR>, dim3(d.nmtiles), dim3(kMassThreads), d.sys, d.mtiles, mask, v, x1);
    };
    static_assert(kMassRMax == 4, "one case per tap count");
    switch (R) {
        case 1: go(std::integral_constant<int, 1>{}); break;
        case 2: go(std::integral_constant<int, 2>{}); break;
        case 3: go(std::integral_constant<int, 3>{}); break;
        default: go(std::integral_constant<int, 4>{}); break;
    }
}
template void launch_mass_sep<double>(const Dev&, int, const zd*, zd*, const int*, hipStream_t);
template void launch_mass_sep<float>(const Dev&, int, const zf*, zf*, const int*, hipStream_t);

}  // namespace apfc
