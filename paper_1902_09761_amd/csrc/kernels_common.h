// Device helpers and launch plumbing shared by the HIP kernel sources of the APFC time step (gfx950,
// CDNA4, wave64).
//
// Every operator here is a constant-coefficient tensor-product stencil of the Q1 element on a
// periodic uniform mesh, built from the 1D weights
//     mass m = h/6 [1 4 1],  stiffness k = 1/h [-1 2 -1],  derivative d = 1/2 [-1 0 1]
// (row = test function, column = trial function), so that
//     M = m (x) m (x) m,   K = sum_d k_d (x) m (x) m,   T_j = 2 sum_d k_{j,d} d_d (x) m (x) m,
//     G_j = -K + i T_j                                  (Sec. II.A, Eq. (8)-(11)).
// The stencils are evaluated separably (x pass, then y, then z) from neighbour loads; all
// kernels stream HBM with 64-wide rows per wave.  Reductions are deterministic: one partial
// per workgroup, summed in a fixed order.
#pragma once

#include "apfc_internal.h"

#include <hip/hip_ext.h>
#include <type_traits>
#include <utility>

namespace apfc {

// ------------------------------------------------------------------------------------------
// complex helpers
// ------------------------------------------------------------------------------------------
template <typename R>
__device__ __forceinline__ cx<R> operator+(cx<R> a, cx<R> b) { return {a.x + b.x, a.y + b.y}; }
template <typename R>
__device__ __forceinline__ cx<R> operator-(cx<R> a, cx<R> b) { return {a.x - b.x, a.y - b.y}; }
template <typename R>
__device__ __forceinline__ cx<R> operator*(R s, cx<R> a) { return {s * a.x, s * a.y}; }
template <typename R>
__device__ __forceinline__ cx<R> cmul(cx<R> a, cx<R> b) { return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x}; }
template <typename R>
__device__ __forceinline__ cx<R> cconj(cx<R> a) { return {a.x, -a.y}; }
template <typename R>
__device__ __forceinline__ R abs2(cx<R> a) { return a.x * a.x + a.y * a.y; }
// conj(a) * b
template <typename R>
__device__ __forceinline__ cx<R> cdot(cx<R> a, cx<R> b) { return {a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x}; }
// i * a
template <typename R>
__device__ __forceinline__ cx<R> mul_i(cx<R> a) { return {-a.y, a.x}; }

template <typename R, typename S>
__device__ __forceinline__ cx<R> ld(const cx<S>* p, long long i) {
    const cx<S> v = p[i];
    return {R(v.x), R(v.y)};
}
// v rounded to precision S (and back): the value a store to cx<S> keeps
template <typename S>
__device__ __forceinline__ zd rounded(zd v) {
    return zd{double(S(v.x)), double(S(v.y))};
}
template <typename S, typename R>
__device__ __forceinline__ void stv(cx<S>* p, long long i, cx<R> v) {
    p[i] = cx<S>{S(v.x), S(v.y)};
}

// ------------------------------------------------------------------------------------------
// reductions
// ------------------------------------------------------------------------------------------
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Sum NV per-thread values over the workgroup; thread 0 receives the totals.  lds >= 4*NV.
template <int NV>
__device__ __forceinline__ void block_sum(double (&v)[NV], double* lds) {
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
    for (int i = 0; i < NV; ++i) {
        const double t = wave_sum(v[i]);
        if (lane == 0) lds[wv * NV + i] = t;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
#pragma unroll
        for (int i = 0; i < NV; ++i) v[i] = ((lds[i] + lds[NV + i]) + lds[2 * NV + i]) + lds[3 * NV + i];
    }
    __syncthreads();
}

// The same fixed-order sum of part[slot*P + t], t in [beg, end), in every workgroup.
template <int NS>
__device__ __forceinline__ void sum_partials(const double* part, long long P, const int (&slot)[NS], int beg,
                                             int end, double (&out)[NS], double* lds) {
    if (threadIdx.x < 64) {
#pragma unroll
        for (int k = 0; k < NS; ++k) {
            double a = 0.0;
            for (int t = beg + (int)threadIdx.x; t < end; t += 64) a += part[slot[k] * P + t];
            a = wave_sum(a);
            if (threadIdx.x == 0) lds[k] = a;
        }
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < NS; ++k) out[k] = lds[k];
    __syncthreads();
}

// The workgroups of one system write their partials, then count themselves on the system's ticket; the
// last one to arrive (device-wide) sees every partial and runs the per-system reduction in the fixed
// order a kernel of its own would, and re-arms the ticket.  No workgroup waits for another.  The
// device-scope release fence this needs writes back the L2, so it is used only where few workgroups
// take part (the second Gram-Schmidt pass, which runs only for systems that need it).
__device__ __forceinline__ bool last_of_system(int* ticket, int si, int n, int* flag_lds) {
    __syncthreads();
    if (threadIdx.x == 0) {
        __threadfence();                      // this workgroup's partials before its ticket
        const int t = atomicAdd(&ticket[si], 1);
        const int last = t == n - 1;
        if (last) ticket[si] = 0;
        *flag_lds = last;
    }
    __syncthreads();
    const bool last = *flag_lds != 0;
    if (last) __threadfence();                // the other workgroups' partials after their tickets
    return last;
}


// ------------------------------------------------------------------------------------------
// geometry: periodic neighbours of node (x, y, z)
// ------------------------------------------------------------------------------------------
template <int DIM>
struct Nbr {
    int xs[3];
    long long rb[DIM == 3 ? 3 : 1][3];   // [dz][dy] local node index of (0, y+dy, z+dz)
};

template <int DIM>
__device__ __forceinline__ void make_nbr(const Sys& s, int x, int y, int z, Nbr<DIM>& n) {
    n.xs[0] = x == 0 ? s.nx - 1 : x - 1;
    n.xs[1] = x;
    n.xs[2] = x == s.nx - 1 ? 0 : x + 1;
    const int ys[3] = {y == 0 ? s.ny - 1 : y - 1, y, y == s.ny - 1 ? 0 : y + 1};
    if constexpr (DIM == 2) {
#pragma unroll
        for (int b = 0; b < 3; ++b) n.rb[0][b] = (long long)ys[b] * s.nx;
    } else {
        const int zs[3] = {z == 0 ? s.nz - 1 : z - 1, z, z == s.nz - 1 ? 0 : z + 1};
#pragma unroll
        for (int c = 0; c < 3; ++c)
#pragma unroll
            for (int b = 0; b < 3; ++b) n.rb[c][b] = ((long long)zs[c] * s.ny + ys[b]) * s.nx;
    }
}

template <int DIM>
__device__ __forceinline__ long long nb_index(const Nbr<DIM>& n, int a, int b, int c) {
    if constexpr (DIM == 2)
        return n.rb[0][b] + n.xs[a];
    else
        return n.rb[c][b] + n.xs[a];
}

// Separable evaluation of (M u, K u, T_j u) at one node; f(a, b, c) returns u at the
// neighbour (x + a - 1, y + b - 1, z + c - 1).
template <int DIM, bool WK, bool WT, typename R, typename F>
__device__ __forceinline__ void stencil(const F& f, R h, R k0, R k1, R k2, cx<R>& Mu, cx<R>& Ku, cx<R>& Tu) {
    const R m0 = h * R(1.0 / 6.0), m1 = h * R(4.0 / 6.0), ih = R(1) / h, half = R(0.5);
    auto mass1 = [&](cx<R> l, cx<R> c, cx<R> r) { return m0 * (l + r) + m1 * c; };
    auto stiff1 = [&](cx<R> l, cx<R> c, cx<R> r) { return ih * ((c + c) - (l + r)); };
    auto der1 = [&](cx<R> l, cx<R> r) { return half * (r - l); };
    if constexpr (DIM == 2) {
        cx<R> mx[3], kx[3], dx[3];
#pragma unroll
        for (int b = 0; b < 3; ++b) {
            const cx<R> l = f(0, b, 1), c = f(1, b, 1), r = f(2, b, 1);
            mx[b] = mass1(l, c, r);
            if (WK) kx[b] = stiff1(l, c, r);
            if (WT) dx[b] = der1(l, r);
        }
        Mu = mass1(mx[0], mx[1], mx[2]);
        if (WK) Ku = mass1(kx[0], kx[1], kx[2]) + stiff1(mx[0], mx[1], mx[2]);
        if (WT) Tu = R(2) * (k0 * mass1(dx[0], dx[1], dx[2]) + k1 * der1(mx[0], mx[2]));
    } else {
        cx<R> mxy[3], kxy[3], dxm[3], dym[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            cx<R> mx[3], kx[3], dx[3];
#pragma unroll
            for (int b = 0; b < 3; ++b) {
                const cx<R> l = f(0, b, c), ce = f(1, b, c), r = f(2, b, c);
                mx[b] = mass1(l, ce, r);
                if (WK) kx[b] = stiff1(l, ce, r);
                if (WT) dx[b] = der1(l, r);
            }
            mxy[c] = mass1(mx[0], mx[1], mx[2]);
            if (WK) kxy[c] = mass1(kx[0], kx[1], kx[2]) + stiff1(mx[0], mx[1], mx[2]);
            if (WT) {
                dxm[c] = mass1(dx[0], dx[1], dx[2]);
                dym[c] = der1(mx[0], mx[2]);
            }
        }
        Mu = mass1(mxy[0], mxy[1], mxy[2]);
        if (WK) Ku = mass1(kxy[0], kxy[1], kxy[2]) + stiff1(mxy[0], mxy[1], mxy[2]);
        if (WT)
            Tu = R(2) * (k0 * mass1(dxm[0], dxm[1], dxm[2]) + k1 * mass1(dym[0], dym[1], dym[2]) +
                         k2 * der1(mxy[0], mxy[2]));
    }
}

// G u = -K u + i T u
template <typename R>
__device__ __forceinline__ cx<R> gop(cx<R> Ku, cx<R> Tu) {
    return {-Ku.x - Tu.y, -Ku.y + Tu.x};
}

// ------------------------------------------------------------------------------------------
// 3D z-marching.  The x and y passes of the separable stencil at one (x, y) column of one plane are
// needed by the three output planes z-1, z, z+1; a thread that walks consecutive planes of its
// column takes them once per plane and keeps the last three in registers, so each input plane is
// used once per field (9 values instead of 27 per node).  The arithmetic is that of stencil().
// zmarch loads the 9 values of a plane from global memory (the operator apply and residual, whose
// basis-vector streams dominate); zmarch_lds stages the planes of the workgroup in LDS (the Chebyshev
// iterations, whose stencil loads dominate).
// ------------------------------------------------------------------------------------------
template <typename R>
struct Plane {
    cx<R> m, k, dx, dy, c;   // over x, y: (m m) u, (k m + m k) u, (d m) u, (m d) u; u at (x, y)
};

template <bool WK, bool WT, typename R, typename F>
__device__ __forceinline__ Plane<R> plane_pass(const F& f, long long base, const int (&xs)[3],
                                               const long long (&rs)[3], R m0, R m1, R ih) {
    const R half = R(0.5);
    cx<R> mx[3], kx[3], dx[3];
    Plane<R> p{};
#pragma unroll
    for (int b = 0; b < 3; ++b) {
        const cx<R> l = f(base + rs[b] + xs[0]), c = f(base + rs[b] + xs[1]), r = f(base + rs[b] + xs[2]);
        mx[b] = m0 * (l + r) + m1 * c;
        if (WK) kx[b] = ih * ((c + c) - (l + r));
        if (WT) dx[b] = half * (r - l);
        if (b == 1) p.c = c;
    }
    p.m = m0 * (mx[0] + mx[2]) + m1 * mx[1];
    if (WK) p.k = (m0 * (kx[0] + kx[2]) + m1 * kx[1]) + ih * ((mx[1] + mx[1]) - (mx[0] + mx[2]));
    if (WT) {
        p.dx = m0 * (dx[0] + dx[2]) + m1 * dx[1];
        p.dy = half * (mx[2] - mx[0]);
    }
    return p;
}

// z pass: (M u, K u, T_j u) at the middle plane from the plane passes of planes z-1, z, z+1.
template <bool WK, bool WT, typename R>
__device__ __forceinline__ void zcombine(const Plane<R>& a, const Plane<R>& b, const Plane<R>& c, R m0, R m1, R ih,
                                         R k0, R k1, R k2, cx<R>& Mu, cx<R>& Ku, cx<R>& Tu) {
    Mu = m0 * (a.m + c.m) + m1 * b.m;
    if (WK) Ku = (m0 * (a.k + c.k) + m1 * b.k) + ih * ((b.m + b.m) - (a.m + c.m));
    if (WT)
        Tu = R(2) * (k0 * (m0 * (a.dx + c.dx) + m1 * b.dx) + k1 * (m0 * (a.dy + c.dy) + m1 * b.dy) +
                     k2 * (R(0.5) * (c.m - a.m)));
}

// Walks planes z0-1 .. z0+RR of column (xc, yc) (periodic), load(f, i) returning node i of field f;
// calls emit(z, P) for the output planes z = z0 .. z0+RR-1 (which may pass nz on a ragged brick),
// P[f][0..2] holding the plane passes of planes z-1, z, z+1.
template <int RR, int NF, bool WK, bool WT, typename R, typename LOAD, typename EMIT>
__device__ __forceinline__ void zmarch(const Sys& s, int xc, int yc, int z0, R m0, R m1, R ih, const LOAD& load,
                                       const EMIT& emit) {
    const int xs[3] = {xc == 0 ? s.nx - 1 : xc - 1, xc, xc == s.nx - 1 ? 0 : xc + 1};
    const long long rs[3] = {(long long)(yc == 0 ? s.ny - 1 : yc - 1) * s.nx, (long long)yc * s.nx,
                             (long long)(yc == s.ny - 1 ? 0 : yc + 1) * s.nx};
    const long long plane = (long long)s.nx * s.ny;
    Plane<R> P[NF][3];
    int zz = z0 == 0 ? s.nz - 1 : z0 - 1;
#pragma unroll
    for (int a = 0; a < RR + 2; ++a) {
        const long long base = zz * plane;
#pragma unroll
        for (int f = 0; f < NF; ++f)
            P[f][2] = plane_pass<WK, WT, R>([&](long long i) { return load(f, i); }, base, xs, rs, m0, m1, ih);
        if (a >= 2) emit(z0 + a - 2, P);
#pragma unroll
        for (int f = 0; f < NF; ++f) {
            P[f][0] = P[f][1];
            P[f][1] = P[f][2];
        }
        zz = zz + 1 == s.nz ? 0 : zz + 1;
    }
}

// zmarch with the next plane loaded while the current one is used: the 9 stored values per field of plane
// z + 1 (ptr(f)[node], type cx<S>) are in flight while the passes of plane z are formed, so a wave has
// arithmetic to issue while its loads are outstanding.  The same operations and emit as zmarch (the
// compiler may contract a few multiply-adds differently).
template <bool WK, bool WT, typename R, typename S>
__device__ __forceinline__ Plane<R> plane_pass_regs(const cx<S> (&u)[9], R m0, R m1, R ih) {
    const R half = R(0.5);
    cx<R> mx[3], kx[3], dx[3];
    Plane<R> p{};
#pragma unroll
    for (int b = 0; b < 3; ++b) {
        const cx<R> l{R(u[3 * b].x), R(u[3 * b].y)}, c{R(u[3 * b + 1].x), R(u[3 * b + 1].y)},
            r{R(u[3 * b + 2].x), R(u[3 * b + 2].y)};
        mx[b] = m0 * (l + r) + m1 * c;
        if (WK) kx[b] = ih * ((c + c) - (l + r));
        if (WT) dx[b] = half * (r - l);
        if (b == 1) p.c = c;
    }
    p.m = m0 * (mx[0] + mx[2]) + m1 * mx[1];
    if (WK) p.k = (m0 * (kx[0] + kx[2]) + m1 * kx[1]) + ih * ((mx[1] + mx[1]) - (mx[0] + mx[2]));
    if (WT) {
        p.dx = m0 * (dx[0] + dx[2]) + m1 * dx[1];
        p.dy = half * (mx[2] - mx[0]);
    }
    return p;
}

template <int RR, int NF, bool WK, bool WT, typename R, typename S, typename PTR, typename EMIT>
__device__ __forceinline__ void zmarch_prefetch(const Sys& s, int xc, int yc, int z0, R m0, R m1, R ih,
                                                const PTR& ptr, const EMIT& emit) {
    const int xs[3] = {xc == 0 ? s.nx - 1 : xc - 1, xc, xc == s.nx - 1 ? 0 : xc + 1};
    const long long rs[3] = {(long long)(yc == 0 ? s.ny - 1 : yc - 1) * s.nx, (long long)yc * s.nx,
                             (long long)(yc == s.ny - 1 ? 0 : yc + 1) * s.nx};
    const long long plane = (long long)s.nx * s.ny;
    cx<S> cur[NF][9], nxt[NF][9];
    auto fetch = [&](long long base, cx<S> (&dst)[NF][9]) {
#pragma unroll
        for (int f = 0; f < NF; ++f)
#pragma unroll
            for (int b = 0; b < 3; ++b)
#pragma unroll
                for (int q = 0; q < 3; ++q) dst[f][3 * b + q] = ptr(f)[base + rs[b] + xs[q]];
    };
    Plane<R> P[NF][3];
    int zz = z0 == 0 ? s.nz - 1 : z0 - 1;
    fetch(zz * plane, cur);
#pragma unroll
    for (int a = 0; a < RR + 2; ++a) {
        const int zn = zz + 1 == s.nz ? 0 : zz + 1;
        if (a + 1 < RR + 2) fetch(zn * plane, nxt);
#pragma unroll
        for (int f = 0; f < NF; ++f) P[f][2] = plane_pass_regs<WK, WT, R, S>(cur[f], m0, m1, ih);
        if (a >= 2) emit(z0 + a - 2, P);
#pragma unroll
        for (int f = 0; f < NF; ++f) {
            P[f][0] = P[f][1];
            P[f][1] = P[f][2];
#pragma unroll
            for (int e = 0; e < 9; ++e) cur[f][e] = nxt[f][e];
        }
        zz = zn;
        // one plane of look-ahead, no more: later planes' loads would hold registers the waves need
        __builtin_amdgcn_sched_barrier(0);
    }
}

// 3D plane march with the planes of the workgroup's 64 x BY columns plus a one-node halo ((64 + 2) x
// (BY + 2)) staged in LDS: the workgroup loads a plane with two coalesced loads per thread and field, the
// next plane while the current one is in use, and every thread takes its x/y pass from LDS (9 LDS reads
// instead of 9 global loads).  buf: [2][NF][(64 + 2) * (BY + 2)] values in the storage type S.
constexpr int kPX = 66, kPY = 6, kPP = kPX * kPY;

template <bool WK, bool WT, typename R, typename S>
__device__ __forceinline__ Plane<R> plane_pass_lds(const cx<S>* b, int lane, int ty, R m0, R m1, R ih) {
    const R half = R(0.5);
    cx<R> mx[3], kx[3], dx[3];
    Plane<R> p{};
#pragma unroll
    for (int q = 0; q < 3; ++q) {
        const cx<S>* row = b + (ty + q) * kPX + lane;
        const cx<R> l{R(row[0].x), R(row[0].y)}, c{R(row[1].x), R(row[1].y)}, r{R(row[2].x), R(row[2].y)};
        mx[q] = m0 * (l + r) + m1 * c;
        if (WK) kx[q] = ih * ((c + c) - (l + r));
        if (WT) dx[q] = half * (r - l);
        if (q == 1) p.c = c;
    }
    p.m = m0 * (mx[0] + mx[2]) + m1 * mx[1];
    if (WK) p.k = (m0 * (kx[0] + kx[2]) + m1 * kx[1]) + ih * ((mx[1] + mx[1]) - (mx[0] + mx[2]));
    if (WT) {
        p.dx = m0 * (dx[0] + dx[2]) + m1 * dx[1];
        p.dy = half * (mx[2] - mx[0]);
    }
    return p;
}

// BY: rows of the brick (the workgroup is 64 x BY threads; planes of (64 + 2) x (BY + 2) nodes in LDS).
template <int BY>
constexpr int kPPb = kPX * (BY + 2);

template <int RR, int NF, bool WK, bool WT, typename R, typename S, int BY = 4, typename LOADG, typename EMIT>
__device__ __forceinline__ void zmarch_lds(const Sys& s, const Tile& tile, int lane, int ty,
                                           cx<S> (*buf)[NF][kPPb<BY>], R m0, R m1, R ih, const LOADG& loadg,
                                           const EMIT& emit) {
    constexpr int NTH = 64 * BY, PP = kPPb<BY>;
    static_assert(PP <= 2 * NTH, "two staged nodes per thread and plane");
    const int e0 = (int)threadIdx.x, e1 = (int)threadIdx.x + NTH;
    auto goff = [&](int e) {
        int gx = (tile.x0 - 1 + e % kPX) % s.nx, gy = (tile.y0 - 1 + e / kPX) % s.ny;
        gx = gx < 0 ? gx + s.nx : gx;
        gy = gy < 0 ? gy + s.ny : gy;
        return (long long)gy * s.nx + gx;
    };
    const long long o0 = goff(e0), o1 = e1 < PP ? goff(e1) : 0;
    const long long plane = (long long)s.nx * s.ny;
    auto fetch = [&](int b, long long base) {
#pragma unroll
        for (int f = 0; f < NF; ++f) {
            buf[b][f][e0] = loadg(f, base + o0);
            if (e1 < PP) buf[b][f][e1] = loadg(f, base + o1);
        }
    };
    Plane<R> P[NF][3];
    int zz = tile.z == 0 ? s.nz - 1 : tile.z - 1;
    fetch(0, zz * plane);
#pragma unroll
    for (int a = 0; a < RR + 2; ++a) {
        __syncthreads();
        const int zn = zz + 1 == s.nz ? 0 : zz + 1;
        if (a + 1 < RR + 2) fetch((a + 1) & 1, zn * plane);
#pragma unroll
        for (int f = 0; f < NF; ++f) P[f][2] = plane_pass_lds<WK, WT, R>(buf[a & 1][f], lane, ty, m0, m1, ih);
        if (a >= 2) emit(tile.z + a - 2, P);
#pragma unroll
        for (int f = 0; f < NF; ++f) {
            P[f][0] = P[f][1];
            P[f][1] = P[f][2];
        }
        zz = zn;
    }
}

// A_j applied at the middle plane of P (field 0: zeta part, field 1: eta part), as apply_A.
template <typename PL>
__device__ __forceinline__ void apply_A_planes(const Sys& s, const PL& P, double m0, double m1, double ih, double dn,
                                               zd& y1, zd& y2) {
    zd Mz, Kz, Tz, Me, Ke, Te;
    zcombine<true, true, double>(P[0][0], P[0][1], P[0][2], m0, m1, ih, s.kv[0], s.kv[1], s.kv[2], Mz, Kz, Tz);
    zcombine<true, true, double>(P[1][0], P[1][1], P[1][2], m0, m1, ih, s.kv[0], s.kv[1], s.kv[2], Me, Ke, Te);
    y1 = Mz - gop(Ke, Te);
    y2 = s.kappa * gop(Kz, Tz) + s.inv_dt * Me + (s.kappa * s.w * dn) * P[1][1].c;
}

// ------------------------------------------------------------------------------------------
// tile iteration.  2D: a workgroup covers x in [x0, x0+64) and rows y0 + ty + 4 r (r < TY/4).
// 3D: a brick x in [x0, x0+64), y = y0 + ty (ty < 4), planes z0 + r (r < TY/4), so a thread walks
// consecutive planes of one (x, y) column (the order the z-marching stencil kernels rely on).
// ------------------------------------------------------------------------------------------
#define TILE_PROLOGUE()                                        \
    const Tile tile = tiles[blockIdx.x];                       \
    if (mask && !mask[tile.sys]) return;                       \
    const Sys s = sys[tile.sys];                               \
    const int x = tile.x0 + (int)(threadIdx.x & 63);           \
    const int ty = (int)(threadIdx.x >> 6);

#define FOR_ROWS(TY)                                                                  \
    _Pragma("unroll") for (int rr_ = 0; rr_ < (TY) / 4; ++rr_)                        \
        if (const int y = DIM == 3 ? tile.y0 + ty : tile.y0 + ty + 4 * rr_,             \
                      pz = DIM == 3 ? tile.z + rr_ : 0;                                 \
            x < s.nx && y < s.ny && pz < s.nz)

// ------------------------------------------------------------------------------------------
// launch plumbing shared by the kernel sources
// ------------------------------------------------------------------------------------------
// records on the device which share of the batch's nodes a masked launch worked on (k_active_frac)
void launch_active_frac(const Sys* sys, int S, const int* mask, double* out, hipStream_t st);

// HIP events around a sampled launch of the probed kernel; after the closing event (outside the timed
// window) k_active_frac records which share of the batch the launch worked on.  A launcher that starts
// its kernel through launch() with ext = true has the two events stamped by the kernel's own dispatch
// (hipExtLaunchKernel), so no event sits between them and the kernel.
struct ProbeScope {
    Probe* p;
    hipStream_t st;
    const Sys* sys;
    int S;
    const int* mask;
    bool on, ext;
    ProbeScope(const Dev& d, int kid, hipStream_t s, double bytes = 0.0, const int* m = nullptr, bool e = false)
        : p(d.probe), st(s), sys(d.sys), S(d.S), mask(m), ext(e) {
        on = p && (p->target == kid || p->target == KID_ALL) && (p->seen[kid]++ % p->every) == 0 &&
             p->n < Probe::kMax;
        if (on) {
            if (!ext) (void)hipEventRecord(p->ev[2 * p->n], st);
            p->bytes[p->n] = bytes;
            p->kid[p->n] = kid;
        }
    }
    template <typename K, typename... A>
    void launch(K kernel, dim3 grid, dim3 block, A... args) {
        if (on && ext)
            hipExtLaunchKernelGGL(kernel, grid, block, 0, st, p->ev[2 * p->n], p->ev[2 * p->n + 1], 0, args...);
        else
            hipLaunchKernelGGL(kernel, grid, block, 0, st, args...);
    }
    ~ProbeScope() {
        if (on) {
            if (!ext) (void)hipEventRecord(p->ev[2 * p->n + 1], st);
            launch_active_frac(sys, S, mask, p->d_frac + p->n, st);
            p->n += 1;
        }
    }
};

template <typename F>
inline void dispatch(const Dev& d, F&& f) {
    auto ty = [&](auto dimc) {
        switch (d.TY) {
            case 4: f(dimc, std::integral_constant<int, 4>{}); break;
            case 8: f(dimc, std::integral_constant<int, 8>{}); break;
            case 32: f(dimc, std::integral_constant<int, 32>{}); break;
            default: f(dimc, std::integral_constant<int, 16>{}); break;
        }
    };
    if (d.dim == 3)
        ty(std::integral_constant<int, 3>{});
    else
        ty(std::integral_constant<int, 2>{});
}

#define TILE_GRID dim3(d.ntiles), dim3(kBlock), 0, st
#define CHUNK_GRID dim3(d.nchunks), dim3(kBlock), 0, st

}  // namespace apfc
