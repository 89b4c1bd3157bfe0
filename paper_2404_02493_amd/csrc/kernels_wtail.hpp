// The small levels of the wave cycle in one workgroup.
//
// Below a few hundred nodes per side every operation of the cycle is a handful
// of microseconds of work, so separate launches are dominated by their latency.
// k_wave_tail runs the whole coarse part of Algorithm 1 from a given level down
// (Chebyshev pre-smoothing, residual + full weighting, the coarser cycle,
// bilinear prolongation, post-smoothing, and the coarsest level's Chebyshev
// iteration) in one workgroup of 1024 threads, with the level arrays in global
// memory and a workgroup barrier between dependent sweeps.  It computes the
// same operations in the same precision as the per-level kernels.
#pragma once

#include "kernels_wave.hpp"

namespace helm {

constexpr int WT_THREADS = 1024;
constexpr int WT_MAXL = 14;

struct TailWaveLevel {
    Geom G;
    int f64;           // arrays of this level are complex128 / double
    const void* n2;
    void* g;
    void* u;
    void* r;
    void* d;
    void* t;
    const double* la;  // device: la[0] = spectral bound of A^* A, la[1] = Chebyshev alpha
};

struct TailWaveArgs {
    TailWaveLevel lv[WT_MAXL + 1];  // indexed by level
    int l0;                         // first level handled here (>= 3)
    int L;
    int cheb_pre, cheb_post, cheb_coarse;
    int level3_literal;
};

// r = A^* (g - A u) (u == nullptr: A^* g), d = r / theta; t holds g - A u.
template <typename P>
__device__ void wt_cheb(const TailWaveLevel& W, bool u_zero, int m, size_t o) {
    const Geom& G = W.G;
    const int n = G.nx;  // nodes per row
    const int N = G.nx * G.ny;
    const P* n2 = (const P*)bsh_one(o, W.n2);
    cplx<P>* g = (cplx<P>*)bsh_one(o, W.g);
    cplx<P>* u = (cplx<P>*)bsh_one(o, W.u);
    cplx<P>* r = (cplx<P>*)bsh_one(o, W.r);
    cplx<P>* d = (cplx<P>*)bsh_one(o, W.d);
    cplx<P>* t = (cplx<P>*)bsh_one(o, W.t);
    const double* la = bsh_one(o, W.la);
    const double lam = la[0], a = lam / la[1];
    const double theta = 0.5 * (lam + a), dc = 0.5 * (lam - a);
    // t = g - A u (or g)
    for (int p = threadIdx.x; p < N; p += WT_THREADS) {
        const int i = p / n, j = p - i * n;
        cplx<P> v{};
        if (i > 0 && j > 0) v = resid_at(G, n2, g, u_zero ? (const cplx<P>*)nullptr : (const cplx<P>*)u, i, j);
        t[p] = v;
        if (u_zero) u[p] = cplx<P>{};
    }
    __syncthreads();
    const P inv_theta = P(1.0 / theta);
    for (int p = threadIdx.x; p < N; p += WT_THREADS) {
        const int i = p / n, j = p - i * n;
        cplx<P> v{};
        if (i > 0 && j > 0) v = applyA_at(G, n2, t, i, j, true);
        r[p] = v;
        d[p] = inv_theta * v;
    }
    __syncthreads();
    double rho = dc / theta;
    for (int step = 1; step <= m; ++step) {
        if (step < m) {
            for (int p = threadIdx.x; p < N; p += WT_THREADS) {  // t = A d
                const int i = p / n, j = p - i * n;
                cplx<P> v{};
                if (i > 0 && j > 0) v = applyA_at(G, n2, d, i, j, false);
                t[p] = v;
            }
            __syncthreads();
            const double den = 2.0 * theta - dc * rho;
            const double rho_new = dc / den;
            const P c1 = P(rho_new * rho), c2 = P(2.0 / den);
            for (int p = threadIdx.x; p < N; p += WT_THREADS) {  // u += d; r -= A^* t; d = c1 d + c2 r
                const int i = p / n, j = p - i * n;
                if (i == 0 || j == 0) continue;
                const cplx<P> dv = d[p];
                const cplx<P> rv = r[p] - applyA_at(G, n2, t, i, j, true);
                u[p] = u[p] + dv;
                r[p] = rv;
                d[p] = c1 * dv + c2 * rv;
            }
            __syncthreads();
            rho = rho_new;
        } else {
            for (int p = threadIdx.x; p < N; p += WT_THREADS) u[p] = u[p] + d[p];
            __syncthreads();
        }
    }
}

// gc = R (g - A u) from level l (precision Pf) to level l + 1 (precision Pc); u may be zero.
template <typename Pf, typename Pc>
__device__ void wt_restrict(const TailWaveLevel& F, const TailWaveLevel& Cl, bool u_zero, size_t o) {
    const Geom& G = F.G;
    const int ncx = G.nx / 2, ncy = G.ny / 2;
    const Pf* n2 = (const Pf*)bsh_one(o, F.n2);
    const cplx<Pf>* g = (const cplx<Pf>*)bsh_one(o, F.g);
    const cplx<Pf>* u = u_zero ? nullptr : (const cplx<Pf>*)bsh_one(o, F.u);
    cplx<Pc>* gc = (cplx<Pc>*)bsh_one(o, Cl.g);
    for (int q = threadIdx.x; q < ncx * ncy; q += WT_THREADS) {
        const int I = q / ncx, J = q - I * ncx;
        cplx<Pf> v{};
        if (I > 0 && J > 0) {
            const int fi = 2 * I, fj = 2 * J;
            auto R = [&](int a, int b) { return resid_at(G, n2, g, u, a, b); };
            const cplx<Pf> c = R(fi, fj);
            const cplx<Pf> ud = ((R(fi - 1, fj) + R(fi + 1, fj)) + R(fi, fj - 1)) + R(fi, fj + 1);
            const cplx<Pf> dg = ((R(fi - 1, fj - 1) + R(fi - 1, fj + 1)) + R(fi + 1, fj - 1)) + R(fi + 1, fj + 1);
            v = Pf(1.0 / 16.0) * ((Pf(4) * c + Pf(2) * ud) + dg);
        }
        gc[q] = ccast<Pc>(v);
    }
    __syncthreads();
}

// u (level l, precision Pf) += P e (level l + 1, precision Pc); u_zero: u = P e.
template <typename Pc, typename Pf>
__device__ void wt_prolong(const TailWaveLevel& F, const TailWaveLevel& Cl, bool u_zero, size_t o) {
    const int n = F.G.nx, ny = F.G.ny;
    cplx<Pf>* u = (cplx<Pf>*)bsh_one(o, F.u);
    const cplx<Pc>* ec = (const cplx<Pc>*)bsh_one(o, Cl.u);
    for (int p = threadIdx.x; p < n * ny; p += WT_THREADS) {
        const int i = p / n, j = p - i * n;
        cplx<Pf> v{};
        if (i > 0 && j > 0) v = prolong_at<Pc, Pf>(ec, n / 2, ny / 2, i, j);
        u[p] = u_zero ? v : u[p] + v;
    }
    __syncthreads();
}

template <typename T>
__device__ void wt_transfer_down(const TailWaveArgs& a, int l, bool u_zero, size_t o) {
    if (a.lv[l + 1].f64) wt_restrict<T, double>(a.lv[l], a.lv[l + 1], u_zero, o);
    else wt_restrict<T, T>(a.lv[l], a.lv[l + 1], u_zero, o);
}
template <typename T>
__device__ void wt_transfer_up(const TailWaveArgs& a, int l, bool u_zero, size_t o) {
    if (a.lv[l + 1].f64) wt_prolong<double, T>(a.lv[l], a.lv[l + 1], u_zero, o);
    else wt_prolong<T, T>(a.lv[l], a.lv[l + 1], u_zero, o);
}

// The cycle on levels l0..L from a zero iterate, as the per-level host recursion runs
// it (no ADR correction here: l0 >= 3).  Levels below L are in precision T (or FP64
// when the whole cycle is FP64); level L is FP64.
template <typename T>
__global__ __launch_bounds__(WT_THREADS) void k_wave_tail(TailWaveArgs a, BatchIdx bi) {
    const size_t o = bi.off();  // the level arrays of this problem (shifted where they are read)
    for (int l = a.l0; l < a.L; ++l) {  // descend: pre-smoothing and restriction
        const bool smooth = l != 3;
        if (smooth) wt_cheb<T>(a.lv[l], true, a.cheb_pre, o);
        wt_transfer_down<T>(a, l, !smooth, o);
    }
    wt_cheb<double>(a.lv[a.L], true, a.cheb_coarse, o);
    for (int l = a.L - 1; l >= a.l0; --l) {  // ascend: prolongation and post-smoothing
        const bool pre = l != 3;
        wt_transfer_up<T>(a, l, !pre, o);
        if (l != 3 || a.level3_literal) wt_cheb<T>(a.lv[l], false, a.cheb_post, o);
    }
}

}  // namespace helm
