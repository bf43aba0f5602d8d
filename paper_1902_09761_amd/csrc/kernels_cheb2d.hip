// The block preconditioner of Eq. (12) with Chebyshev-Jacobi inner solves, fused per step on LDS regions
// (2D), for gfx950, with its launcher.
#include "kernels_common.h"

namespace apfc {

// ------------------------------------------------------------------------------------------
// Block preconditioner with Chebyshev-Jacobi inner solves, fused per step (2D).
//
// A workgroup owns a region of RX x RY nodes = an interior tile plus `halo` layers (periodic wrap).
// Every stencil application inside the region is evaluated from the region's values (staged in LDS, or,
// for FP32 regions one wave wide, held in registers with the edge rows of the waves exchanged through
// LDS) and is exact one layer further in than the previous one, so after `halo` applications the interior
// holds the same values an unfused sweep over the whole mesh would give.  Stages 0 and 1 can also form
// their half of the next FGMRES basis vector as they load it (VIn).  Three kernels per preconditioner
// application:
//   STAGE 0: x1   = Cheb_M^{sM}(beta1)                         (step 1)
//   STAGE 1: x2   = Cheb_L^{sL}(beta2 - kappa G x1)             (step 2)
//   STAGE 2: chi2 = Cheb_L^{sL}(M x2);  chi1 = x1 - (x2 - chi2/sqrt(dt))/sqrt(kappa)   (steps 3, 4)
// Chebyshev iteration for D^{-1} A with spectrum in [theta - delta, theta + delta], x0 = 0
// (three-term recurrence on the correction d):
//   d0 = r0/(theta D), rho0 = delta/theta; x_{k+1} = x_k + d_k;
//   r_{k+1} = r_k - A d_k; rho_{k+1} = 1/(2 theta/delta - rho_k);
//   d_{k+1} = rho_{k+1} rho_k d_k + (2 rho_{k+1}/delta) D^{-1} r_{k+1}.
// The spectral bounds are exact for the constant-coefficient operators (symbol extremes at the
// corners cos(theta_d) = +-1), so the iteration needs no inner products.
// ------------------------------------------------------------------------------------------
__device__ __forceinline__ int wrapi(int g, int n) {
    g %= n;
    return g < 0 ? g + n : g;
}

// Whole-wave lane shifts by one lane (DPP wave_shr:1 / wave_shl:1): after lane_shift<kDppWaveShr1>, lane i
// holds lane i - 1's value (lane 0 gets 0); after kDppWaveShl1, lane i + 1's (lane 63 gets 0).
constexpr int kDppWaveShl1 = 0x130, kDppWaveShr1 = 0x138;
template <int CTRL>
__device__ __forceinline__ float lane_shift(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xf, 0xf, false));
}
template <int CTRL>
__device__ __forceinline__ double lane_shift(double v) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffffLL), CTRL, 0xf, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xf, 0xf, false);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
template <int CTRL, typename T>
__device__ __forceinline__ cx<T> lane_shift(cx<T> v) {
    return cx<T>{lane_shift<CTRL>(v.x), lane_shift<CTRL>(v.y)};
}

// The operators of the inner solves in split form.  With P = [1 4 1], Q = [-1 2 -1] = 6 delta - P and
// E = [-1 0 1], the bilinear element stencils are M = (h/6)^2 P(x)P,
// K = (1/6)(Q(x)P + P(x)Q) = (delta(x)P + P(x)delta) - P(x)P/3 and T_j = (h/6)(k0 E(x)P + k1 P(x)E).
// At a node with rows A, B, C (y - 1, y, y + 1), x passes p = P u and e = E u of those rows and centre
// values uA, uB, uC:
//   (cM M + cK K) u = a (pA + pC) + b pB + c (uA + uC) + d uB,
//   a = cM (h/6)^2 - cK/3,  b = 4 a + cK,  c = cK,  d = 4 cK   (M alone: a = (h/6)^2, b = 4 a, c = d = 0),
//   T_j u = (h/6) (k0 (eA + 4 eB + eC) + k1 (pC - pA)).
// The LDS region keeps one pad row above and below the RY region rows (region row q at LDS row q + 1),
// so a thread's rows r0 - 1 .. r0 + NP are rows of the array with no clamping and every load of the
// sweep is a fixed offset from the thread's three column addresses.  split_sweep streams them (b = LDS row
// r0 of the buffer, i.e. region row r0 - 1; columns xm, xc, xp) and calls
// f(i, pA, pB, pC, uA, uB, uC, eA, eB, eC) for region row r0 + i (e only with WE).  The loads of the next
// row are issued while the current one is used, and no further (a scheduling barrier per row): hoisting
// every row's loads ahead would cost registers the workgroups of a CU need.
template <typename T, int NP, int RX, bool WE, typename F>
__device__ __forceinline__ void split_sweep(const cx<T>* b, int xm, int xc, int xp, F&& f) {
    const cx<T> zero{T(0), T(0)};
    cx<T> pA = zero, pB = zero, uA = zero, uB = zero, eA = zero, eB = zero;
    const cx<T>* bm = b + xm;
    const cx<T>* bc = b + xc;
    const cx<T>* bp = b + xp;
    cx<T> l = bm[0], c = bc[0], r = bp[0];
#pragma unroll
    for (int a = 0; a < NP + 2; ++a) {
        cx<T> ln = zero, cn = zero, rn = zero;
        if (a + 1 < NP + 2) {
            ln = bm[(a + 1) * RX];
            cn = bc[(a + 1) * RX];
            rn = bp[(a + 1) * RX];
        }
        const cx<T> pC = T(4) * c + (l + r);
        const cx<T> eC = WE ? r - l : zero;
        if (a >= 2) f(a - 2, pA, pB, pC, uA, uB, c, eA, eB, eC);
        pA = pB; pB = pC;
        uA = uB; uB = c;
        eA = eB; eB = eC;
        l = ln; c = cn; r = rn;
        __builtin_amdgcn_sched_barrier(0);
    }
}

// split_sweep for regions one wave wide (RX = 64, the thread's lane is its column) with the thread's NP
// rows u[] in registers: the x neighbours come by lane shifts (0 beyond the region's outer columns, whose
// values only reach the halo), the rows above and below the thread's block from the neighbouring waves
// through edge[w][0] and edge[w][1] (first and last row of the block of wave w; 0 above the first block and
// below the last, as the pad rows of the LDS region).  One barrier, after the edge rows are stored.
// f(i, ...) is called as by split_sweep, in row order, and may overwrite u[i] (read by then).
template <typename T, int NP, int NW, bool WE, typename F>
__device__ __forceinline__ void reg_sweep(cx<T> (&u)[NP], cx<T> (*edge)[2][kTX], int w, F&& f) {
    const int lane = (int)threadIdx.x & (kTX - 1);
    edge[w][0][lane] = u[0];
    edge[w][1][lane] = u[NP - 1];
    __syncthreads();
    const cx<T> zero{T(0), T(0)};
    const cx<T> above = w > 0 ? edge[w - 1][1][lane] : zero;
    const cx<T> below = w + 1 < NW ? edge[w + 1][0][lane] : zero;
    auto xpass = [&](cx<T> c, cx<T>& p, cx<T>& e) {
        const cx<T> l = lane_shift<kDppWaveShr1>(c), r = lane_shift<kDppWaveShl1>(c);
        p = T(4) * c + (l + r);
        e = WE ? r - l : zero;
    };
    cx<T> uA = above, uB = u[0], pA, pB, eA, eB;
    xpass(uA, pA, eA);
    xpass(uB, pB, eB);
#pragma unroll
    for (int i = 0; i < NP; ++i) {
        const cx<T> uC = i + 1 < NP ? u[i + 1] : below;
        cx<T> pC, eC;
        xpass(uC, pC, eC);
        f(i, pA, pB, pC, uA, uB, uC, eA, eB, eC);
        uA = uB;
        uB = uC;
        pA = pB;
        pB = pC;
        eA = eB;
        eB = eC;
    }
}

struct SplitCoef {
    double a, b, c, d;
};
__host__ __device__ inline SplitCoef split_coef(double h, double cM, double cK) {
    const double m = (h / 6.0) * (h / 6.0), a = cM * m - cK / 3.0;
    return {a, 4.0 * a + cK, cK, 4.0 * cK};
}

// Global node of the thread's region rows: x wrapped once per thread, rows walked with a running
// periodic row index (no division per row).
struct RegionRows {
    long long base, gx;
    int gy, nx, ny;
    __device__ __forceinline__ long long at() const { return base + (long long)gy * nx + gx; }
    __device__ __forceinline__ void next() { gy = gy + 1 == ny ? 0 : gy + 1; }
};

// FP32 (mixed precision): two region buffers used in turn; iteration k reads the correction d_{k-1} from
// one and writes d_k into the other as soon as it is formed, so each iteration needs one barrier and d_k
// needs no registers (a thread's own d_{k-1} is the centre value of its sweep).  FP64 regions are twice
// as large: one buffer, d_k kept in registers until the sweep has finished reading.
template <typename T>
constexpr int cheb_buffers() { return sizeof(T) == 4 ? 2 : 1; }

// MR > 0 (stage 0 only): x1 = W beta1 with the separable mass inverse of MR taps per side (Sys::wsep; the
// operator of launch_mass_sep) instead of the Chebyshev mass iterations: an x filter of the region's rows,
// then a y filter at the thread's rows.
template <typename T, int STAGE, int RX, int RY, int NTH, int MR = 0>
__global__ __launch_bounds__(NTH, sizeof(T) == 4 ? 4 : 2) void k_cheb2d(
    const Sys* sys, const CTile* tiles, const int* mask, const cx<T>* v, cx<T>* x1, cx<T>* x2, cx<T>* z, int sM,
    int sL, int halo, long long NT, VIn<T> vin) {
    // the separable stage 0 needs one region buffer: half the LDS, twice the workgroups per CU
    constexpr int NB = MR > 0 ? 1 : cheb_buffers<T>();
    constexpr int RL = RY + 2, RP = RX * RL, NP = RX * RY / NTH;
    static_assert((RX * RY) % NTH == 0 && NTH % RX == 0, "region rows must map onto whole workgroup rows");
    // RG: the Chebyshev stages of FP32 regions one wave wide keep the thread's rows in registers
    // (reg_sweep); the region is not staged in LDS, only the edge rows of the waves' blocks (two sets, used
    // in turn by consecutive sweeps, so each sweep needs one barrier)
    constexpr bool RG = MR == 0 && RX == kTX && sizeof(T) == 4;
    constexpr int NW = NTH / RX;
    __shared__ cx<T> bufs[RG ? 1 : NB][RG ? 1 : RP];
    __shared__ cx<T> edges[RG ? 2 : 1][RG ? NW : 1][2][kTX];
    const int wv = (int)threadIdx.x / RX;
    const CTile tile = tiles[blockIdx.x];
    if (mask && !mask[tile.sys]) return;
    const Sys s = sys[tile.sys];
    const int IX = RX - 2 * halo, IY = RY - 2 * halo;
    // thread -> region column px and NP consecutive rows r0 .. r0 + NP - 1
    const int px = threadIdx.x % RX, r0 = (threadIdx.x / RX) * NP;
    const int xm = px > 0 ? px - 1 : px, xp = px < RX - 1 ? px + 1 : px;
    const RegionRows rows0{s.off, (long long)wrapi(tile.x0 - halo + px, s.nx), wrapi(tile.y0 - halo + r0, s.ny), s.nx,
                           s.ny};
    auto lrow = [&](cx<T>* b, int i) -> cx<T>& { return b[(r0 + 1 + i) * RX + px]; };
    // the pad rows only feed the outermost halo rows; zero them so that no stale value is ever read
    if constexpr (!RG)
        for (int e = threadIdx.x; e < RX; e += NTH)
#pragma unroll
            for (int q = 0; q < NB; ++q) {
                bufs[q][e] = cx<T>{T(0), T(0)};
                bufs[q][(RL - 1) * RX + e] = cx<T>{T(0), T(0)};
            }
    cx<T> X[NP], R[NP];
    constexpr int PC = NP % 4 == 0 ? 4 : NP % 3 == 0 ? 3 : NP % 2 == 0 ? 2 : 1;
    // nodes the region owns (its interior; no wrap: each mesh node is owned by exactly one region)
    const int ix = px - halo;
    const bool own_x = ix >= 0 && ix < IX && tile.x0 + ix < s.nx;
    auto own_row = [&](int i) {
        const int iy = r0 + i - halo;
        return iy >= 0 && iy < IY && tile.y0 + iy < s.ny;
    };
    // The input half at offset hoff into R: v, or the basis vector formed from vin (normalised, and projected
    // against the earlier basis vectors, here instead of in a pass of its own), whose owned nodes are also
    // stored to vin.vout
    auto load_in = [&](long long hoff) {
        RegionRows g = rows0;
        if (!vin.src) {
#pragma unroll
            for (int i = 0; i < NP; ++i, g.next()) R[i] = v[hoff + g.at()];
            return;
        }
        const double* hc = vin.hcoef + (long long)tile.sys * vin.hld;
        const double sc = vin.scale[tile.sys];
        // PC rows at a time: FP64 accumulators for all NP rows would cost a third of the workgroups per CU
#pragma unroll
        for (int i0 = 0; i0 < NP; i0 += PC) {
            zd u[PC];
            long long gi[PC];
#pragma unroll
            for (int i = 0; i < PC; ++i, g.next()) {
                gi[i] = hoff + g.at();
                u[i] = ld<double>(vin.src, gi[i]);
            }
            for (int l = 0; l < vin.nv; ++l) {
                const zd c{hc[2 * l], hc[2 * l + 1]};
                const cx<T>* Vl = vin.V + l * vin.vs;
#pragma unroll
                for (int i = 0; i < PC; ++i) u[i] = u[i] - cmul(c, ld<double>(Vl, gi[i]));
            }
#pragma unroll
            for (int i = 0; i < PC; ++i) {
                R[i0 + i] = cx<T>{T(sc * u[i].x), T(sc * u[i].y)};
                if (own_x && own_row(i0 + i)) vin.vout[gi[i]] = R[i0 + i];
            }
        }
    };
    // right-hand side of the inner solve
    if constexpr (STAGE == 0) {
        load_in(0);
    } else {
        // stage 1: r = beta2 - kappa G x1 with G = -K + i T_j (r += kappa K x1 - i kappa T_j x1); stage 2: r = M x2
        const T k3 = T(s.kappa / 3.0), k4 = T(4.0 * s.kappa), kap = T(s.kappa);
        const T g0 = T(s.kappa * s.h / 6.0 * s.kv[0]), g1 = T(s.kappa * s.h / 6.0 * s.kv[1]);
        const SplitCoef m = split_coef(s.h, 1.0, 0.0);
        const T ma = T(m.a), mb = T(m.b);
        auto rhs = [&](int i, cx<T> pA, cx<T> pB, cx<T> pC, cx<T> uA, cx<T> uB, cx<T> uC, cx<T> eA, cx<T> eB,
                       cx<T> eC) {
            if constexpr (STAGE == 1) {
                const cx<T> kk = kap * (uA + uC) + k4 * uB - k3 * ((pA + pC) + pB);
                const cx<T> tt = g0 * (T(4) * eB + (eA + eC)) + g1 * (pC - pA);
                R[i] = R[i] + cx<T>{kk.x + tt.y, kk.y - tt.x};
            } else {
                R[i] = ma * (pA + pC) + mb * pB;
            }
        };
        if constexpr (RG) {
            cx<T> U[NP];
            RegionRows g = rows0;
#pragma unroll
            for (int i = 0; i < NP; ++i, g.next()) U[i] = STAGE == 1 ? x1[g.at()] : x2[g.at()];
            if constexpr (STAGE == 1) load_in(NT);
            reg_sweep<T, NP, NW, STAGE == 1>(U, edges[0], wv, rhs);
        } else {
            {
                RegionRows g = rows0;
#pragma unroll
                for (int i = 0; i < NP; ++i, g.next()) lrow(bufs[0], i) = STAGE == 1 ? x1[g.at()] : x2[g.at()];
            }
            if constexpr (STAGE == 1) load_in(NT);
            __syncthreads();
            split_sweep<T, NP, RX, STAGE == 1>(bufs[0] + r0 * RX, xm, px, xp, rhs);
        }
    }
    static_assert(MR == 0 || (STAGE == 0 && MR <= kMassRMax), "the separable mass inverse is step 1");
    if constexpr (MR > 0 && RX == kTX) {
        // a region row is one wave: the x filter by lane shifts (DPP) in registers; the y filter from the
        // thread's own rows, and from LDS for the MR rows beyond either end of its block, which the waves
        // above and below store.  Rows q in [MR, RY - MR) and columns in [MR, RX - MR) come out exact.
        static_assert(2 * MR <= NP, "a thread's block holds the rows its neighbours need");
        T w[MR + 1];
#pragma unroll
        for (int k = 0; k <= MR; ++k) w[k] = T(s.wsep[k]);
#pragma unroll
        for (int i = 0; i < NP; ++i) {
            cx<T> lo = R[i], hi = R[i];
            cx<T> acc = w[0] * R[i];
#pragma unroll
            for (int k = 1; k <= MR; ++k) {
                lo = lane_shift<kDppWaveShr1>(lo);   // column px - k
                hi = lane_shift<kDppWaveShl1>(hi);   // column px + k
                acc = acc + w[k] * (lo + hi);
            }
            X[i] = acc;
        }
#pragma unroll
        for (int i = 0; i < NP; ++i)
            if (i < MR || i >= NP - MR) lrow(bufs[0], i) = X[i];
        __syncthreads();
        // (R, no longer needed, takes the y-filtered rows)
#pragma unroll
        for (int i = 0; i < NP; ++i) {
            cx<T> acc = w[0] * X[i];
#pragma unroll
            for (int k = 1; k <= MR; ++k) {
                const cx<T> a = i - k >= 0 ? X[i - k] : lrow(bufs[0], i - k);
                const cx<T> b = i + k < NP ? X[i + k] : lrow(bufs[0], i + k);
                acc = acc + w[k] * (a + b);
            }
            R[i] = acc;
        }
#pragma unroll
        for (int i = 0; i < NP; ++i) X[i] = R[i];
    } else if constexpr (MR > 0) {
        // x filter of the thread's rows from LDS into X, written back over the region (one buffer), then the
        // y filter; region rows q in [MR, RY - MR) and columns in [MR, RX - MR) come out exact, and the
        // interior lies inside them (halo >= MR)
        T w[MR + 1];
#pragma unroll
        for (int k = 0; k <= MR; ++k) w[k] = T(s.wsep[k]);
#pragma unroll
        for (int i = 0; i < NP; ++i) lrow(bufs[0], i) = R[i];
        __syncthreads();
        const bool xin = px >= MR && px < RX - MR;
#pragma unroll
        for (int i = 0; i < NP; ++i) {
            const cx<T>* row = &lrow(bufs[0], i);
            cx<T> acc = cx<T>{T(0), T(0)};
            if (xin) {
                acc = w[0] * row[0];
#pragma unroll
                for (int k = 1; k <= MR; ++k) acc = acc + w[k] * (row[-k] + row[k]);
            }
            X[i] = acc;
        }
        __syncthreads();
#pragma unroll
        for (int i = 0; i < NP; ++i) lrow(bufs[0], i) = X[i];
        __syncthreads();
#pragma unroll
        for (int i = 0; i < NP; ++i) {
            const int q = r0 + i;
            if (q < MR || q >= RY - MR) continue;
            const cx<T>* col = &lrow(bufs[0], i);
            cx<T> acc = w[0] * col[0];
#pragma unroll
            for (int k = 1; k <= MR; ++k) acc = acc + w[k] * (col[-k * RX] + col[k * RX]);
            X[i] = acc;
        }
    } else {
    // Chebyshev iterations on OP = M (stage 0) or L (stages 1, 2)
    constexpr bool isM = STAGE == 0;
    const int its = isM ? sM : sL;
    const double(*cb)[2] = sys[tile.sys].cb[isM ? 0 : 1];
    const SplitCoef oc = split_coef(s.h, isM ? 1.0 : s.isq_dt, isM ? 0.0 : s.sq_kap);
    const T oa = T(oc.a), ob = T(oc.b), occ = T(oc.c), od = T(oc.d);
    const T d0 = T(cb[0][0]);
    if constexpr (RG) {
        // d_{k-1} of the thread's rows in D; iteration k sweeps them with edge set k & 1 (set 0 also served
        // the right-hand side sweep of stages 1 and 2, whose reads finished before iteration 1's barrier) and
        // replaces each row's d once the sweep has read it
        cx<T> D[NP];
#pragma unroll
        for (int i = 0; i < NP; ++i) {
            D[i] = d0 * R[i];
            X[i] = D[i];
        }
        auto iteration = [&](int k, auto store) {
            const T c1 = T(cb[k][0]), c2 = T(cb[k][1]);
            reg_sweep<T, NP, NW, false>(D, edges[k & 1], wv, [&](int i, cx<T> pA, cx<T> pB, cx<T> pC, cx<T> uA,
                                                                  cx<T> uB, cx<T> uC, cx<T>, cx<T>, cx<T>) {
                cx<T> q = R[i] - oa * (pA + pC) - ob * pB;
                if constexpr (!isM) q = q - occ * (uA + uC) - od * uB;
                R[i] = q;
                const cx<T> dv = c1 * uB + c2 * q;
                X[i] = X[i] + dv;
                if constexpr (decltype(store)::value) D[i] = dv;
            });
        };
        for (int k = 1; k + 1 < its; ++k) iteration(k, std::true_type{});
        if (its > 1) iteration(its - 1, std::false_type{});
    } else if constexpr (NB == 2) {
        // d_0 into bufs[1]; iteration k reads d_{k-1} from bufs[k & 1] (the barrier at its start orders it
        // after every write of d_{k-1} and after every read of the buffer it writes, bufs[(k + 1) & 1], by
        // iteration k - 1 or by the prologue of stages 1 and 2)
#pragma unroll
        for (int i = 0; i < NP; ++i) {
            const cx<T> dv = d0 * R[i];
            X[i] = dv;
            lrow(bufs[1], i) = dv;
        }
        auto iteration = [&](int k, auto store) {
            __syncthreads();
            const cx<T>* b = bufs[k & 1];
            cx<T>* bn = bufs[(k + 1) & 1];
            const T c1 = T(cb[k][0]), c2 = T(cb[k][1]);
            split_sweep<T, NP, RX, false>(b + r0 * RX, xm, px, xp, [&](int i, cx<T> pA, cx<T> pB, cx<T> pC, cx<T> uA,
                                                                        cx<T> uB, cx<T> uC, cx<T>, cx<T>, cx<T>) {
                // r -= OP d_{k-1} (uB = this node's d_{k-1}), as a chain of fused multiply-adds (the mass
                // operator has no centre terms); d_k = c1 d_{k-1} + c2 r; x += d_k
                cx<T> q = R[i] - oa * (pA + pC) - ob * pB;
                if constexpr (!isM) q = q - occ * (uA + uC) - od * uB;
                R[i] = q;
                const cx<T> dv = c1 * uB + c2 * q;
                X[i] = X[i] + dv;
                if constexpr (decltype(store)::value) lrow(bn, i) = dv;
            });
        };
        // the last iteration's d is not needed by anyone: it is not stored
        for (int k = 1; k + 1 < its; ++k) iteration(k, std::true_type{});
        if (its > 1) iteration(its - 1, std::false_type{});
    } else {
        cx<T> Dd[NP];
#pragma unroll
        for (int i = 0; i < NP; ++i) {
            Dd[i] = d0 * R[i];
            X[i] = Dd[i];
        }
        for (int k = 1; k < its; ++k) {
            __syncthreads();
#pragma unroll
            for (int i = 0; i < NP; ++i) lrow(bufs[0], i) = Dd[i];
            __syncthreads();
            const T c1 = T(cb[k][0]), c2 = T(cb[k][1]);
            split_sweep<T, NP, RX, false>(bufs[0] + r0 * RX, xm, px, xp,
                                          [&](int i, cx<T> pA, cx<T> pB, cx<T> pC, cx<T> uA, cx<T> uB, cx<T> uC,
                                              cx<T>, cx<T>, cx<T>) {
                                              cx<T> q = R[i] - oa * (pA + pC) - ob * pB;
                                              if constexpr (!isM) q = q - occ * (uA + uC) - od * uB;
                                              R[i] = q;
                                              Dd[i] = c1 * Dd[i] + c2 * R[i];
                                              X[i] = X[i] + Dd[i];
                                          });
        }
    }
    }
    // output at the owned nodes
    if (!own_x) return;
    RegionRows g = rows0;
#pragma unroll
    for (int i = 0; i < NP; ++i, g.next()) {
        if (!own_row(i)) continue;
        const long long gi = g.at();
        if constexpr (STAGE == 0) {
            x1[gi] = X[i];
        } else if constexpr (STAGE == 1) {
            x2[gi] = X[i];
        } else {
            const cx<T> chi2 = X[i];
            z[gi] = x1[gi] - T(s.isq_kap) * (x2[gi] - T(s.isq_dt) * chi2);
            z[NT + gi] = chi2;
        }
    }
}

template <typename T, int RX, int RY, int NTH>
static void cheb_stages(const Dev& d, const CTile* ctiles, int nctiles, int halo, const cx<T>* v, cx<T>* z,
                        cx<T>* x1, cx<T>* x2, int mass_iters, int diff_iters, int mass_sep, const VIn<T>& vin,
                        const int* mask, hipStream_t st) {
    const dim3 g(nctiles), b(NTH);
    // input half read (v, or the vectors the basis vector is formed from) and then the basis vector written
    const double pts = (double)d.NT, in = (double)sizeof(cx<T>) * (vin.src ? 1 + vin.nv : 1),
                 vb = vin.src ? (double)sizeof(cx<T>) : 0.0;
    {
        ProbeScope ps(d, KID_CHEB, st, pts * (in + sizeof(cx<T>) + vb), mask, true);
        auto stage0 = [&](auto mr) {
            ps.launch(k_cheb2d<T, 0, RX, RY, NTH, decltype(mr)::value>, g, b, d.sys, ctiles, mask, v, x1, x2, z,
                      mass_iters, diff_iters, halo, d.NT, vin);
        };
        static_assert(kMassRMax == 4, "one case per tap count");
        switch (mass_sep) {
            case 0: stage0(std::integral_constant<int, 0>{}); break;
            case 1: stage0(std::integral_constant<int, 1>{}); break;
            case 2: stage0(std::integral_constant<int, 2>{}); break;
            case 3: stage0(std::integral_constant<int, 3>{}); break;
            default: stage0(std::integral_constant<int, 4>{}); break;
        }
    }
    {
        ProbeScope ps(d, KID_CHEB, st, pts * (in + 2 * sizeof(cx<T>) + vb), mask, true);
        ps.launch(k_cheb2d<T, 1, RX, RY, NTH>, g, b, d.sys, ctiles, mask, v, x1, x2, z, mass_iters, diff_iters, halo,
                  d.NT, vin);
    }
    ProbeScope ps(d, KID_CHEB, st, pts * 4 * sizeof(cx<T>), mask, true);
    ps.launch(k_cheb2d<T, 2, RX, RY, NTH>, g, b, d.sys, ctiles, mask, v, x1, x2, z, mass_iters, diff_iters, halo,
              d.NT, VIn<T>{});
}

template <typename T>
void launch_precond_cheb(const Dev& d, int shape, const CTile* ctiles, int nctiles, int halo, const cx<T>* v,
                         cx<T>* z, cx<T>* x1, cx<T>* x2, int mass_iters, int diff_iters, int mass_sep,
                         const VIn<T>& vin, const int* mask, hipStream_t st) {
#define APFC_CHEB_SHAPE(I)                                                                                       \
    case I:                                                                                                      \
        cheb_stages<T, kChebShape[I][0], kChebShape[I][1], kChebShape[I][2]>(                                    \
            d, ctiles, nctiles, halo, v, z, x1, x2, mass_iters, diff_iters, mass_sep, vin, mask, st);               \
        break;
    static_assert(kChebShapes == 6, "one case per region shape");
    switch (shape) {
        APFC_CHEB_SHAPE(1)
        APFC_CHEB_SHAPE(2)
        APFC_CHEB_SHAPE(3)
        APFC_CHEB_SHAPE(4)
        APFC_CHEB_SHAPE(5)
        default: cheb_stages<T, kChebShape[0][0], kChebShape[0][1], kChebShape[0][2]>(
            d, ctiles, nctiles, halo, v, z, x1, x2, mass_iters, diff_iters, mass_sep, vin, mask, st);
    }
#undef APFC_CHEB_SHAPE
}
template void launch_precond_cheb<double>(const Dev&, int, const CTile*, int, int, const zd*, zd*, zd*, zd*, int, int,
                                          int, const VIn<double>&, const int*, hipStream_t);
template void launch_precond_cheb<float>(const Dev&, int, const CTile*, int, int, const zf*, zf*, zf*, zf*, int, int,
                                         int, const VIn<float>&, const int*, hipStream_t);

}  // namespace apfc
