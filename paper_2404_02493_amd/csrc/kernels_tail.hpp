// Single-workgroup kernels for the small levels of a hierarchy.
//
// Below about 128 x 128 nodes a level is too small to fill the GPU and every
// launch costs more than the work it carries.  These kernels run the whole
// bottom part of a V-cycle in one workgroup of 1024 threads: vectors stay in
// global memory (they are a few hundred KB and L2-resident), scalars and the
// Hessenberg matrix live in LDS, and __syncthreads orders the passes.
#pragma once

#include "kernels_sstep.hpp"

namespace helm {

constexpr int TB_MAX = 1024;      // largest tail workgroup
constexpr int TW_MAX = TB_MAX / 64;
constexpr int TAIL_LEVELS = 6;    // at most this many levels in a tail

template <typename T>
struct AdrTailLevel {
    AdrGeom A;
    const T* px;
    const T* py;
    const cplx<T>* c0;
    cplx<T>* b;
    cplx<T>* x;
    cplx<T>* V[MAXM + 1];
    int m;  // GMRES dimension on this level
};

template <typename T>
struct AdrTailArgs {
    AdrTailLevel<T> lv[TAIL_LEVELS];
    int nlev;  // levels lv[0] (finest of the tail) .. lv[nlev-1] (coarsest ADR level)
};

// Block-wide sums of K values; every thread receives them in out[] (LDS).
template <int K, int TB>
__device__ __forceinline__ void tail_sum(const double (&acc)[K], int kcount, double* red, double* out) {
    constexpr int TW = TB / 64;
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
#pragma unroll
    for (int v = 0; v < K; ++v) {
        if (v < kcount) {
            double s = wave_sum(acc[v]);
            if (lane == 0) red[wave * K + v] = s;
        }
    }
    __syncthreads();
    if (tid < kcount) {
        double s = 0.0;
#pragma unroll
        for (int w = 0; w < TW; ++w) s += red[w * K + tid];
        out[tid] = s;
    }
    __syncthreads();
}

// Hessenberg least squares with complex Givens rotations (thread 0, LDS data).
// H(i,j) at H[2*(i + j*(MAXM+1))]; y receives cols complex values.
__device__ inline void tail_lsq(double* H, double beta, int cols, double* y, double* e) {
    auto Hp = [&](int i, int j) { return H + 2 * (i + j * (MAXM + 1)); };
    for (int i = 0; i <= cols; ++i) e[2 * i] = e[2 * i + 1] = 0.0;
    e[0] = beta;
    for (int j = 0; j < cols; ++j) {
        double ar = Hp(j, j)[0], ai = Hp(j, j)[1];
        double br = Hp(j + 1, j)[0], bi = Hp(j + 1, j)[1];
        double na = hypot(ar, ai), nb = hypot(br, bi);
        double c, sr, si;
        if (nb == 0.0) {
            c = 1.0; sr = 0.0; si = 0.0;
        } else if (na == 0.0) {
            c = 0.0; sr = 1.0; si = 0.0;
        } else {
            double rho = hypot(na, nb);
            c = na / rho;
            double ur = ar / na, ui = ai / na;
            sr = (ur * br + ui * bi) / rho;
            si = (ui * br - ur * bi) / rho;
        }
        for (int q = j; q < cols; ++q) {
            double xr = Hp(j, q)[0], xi = Hp(j, q)[1];
            double yr = Hp(j + 1, q)[0], yi = Hp(j + 1, q)[1];
            Hp(j, q)[0] = c * xr + (sr * yr - si * yi);
            Hp(j, q)[1] = c * xi + (sr * yi + si * yr);
            Hp(j + 1, q)[0] = -(sr * xr + si * xi) + c * yr;
            Hp(j + 1, q)[1] = -(sr * xi - si * xr) + c * yi;
        }
        double xr = e[2 * j], xi = e[2 * j + 1];
        e[2 * j] = c * xr;
        e[2 * j + 1] = c * xi;
        e[2 * j + 2] = -(sr * xr + si * xi);
        e[2 * j + 3] = -(sr * xi - si * xr);
    }
    for (int i = cols - 1; i >= 0; --i) {
        double accr = e[2 * i], acci = e[2 * i + 1];
        for (int q = i + 1; q < cols; ++q) {
            double hr_ = Hp(i, q)[0], hi_ = Hp(i, q)[1];
            accr -= hr_ * y[2 * q] - hi_ * y[2 * q + 1];
            acci -= hr_ * y[2 * q + 1] + hi_ * y[2 * q];
        }
        double dr = Hp(i, i)[0], di = Hp(i, i)[1];
        double d = dr * dr + di * di;
        y[2 * i] = (accr * dr + acci * di) / d;
        y[2 * i + 1] = (acci * dr - accr * di) / d;
    }
}

// LDS state of the in-block GMRES.
struct TailLds {
    double red[TW_MAX * 2 * (MAXM + 1)];
    double sums[2 * (MAXM + 1)];
    double cq[2 * (MAXM + 1)];
    double H[2 * (MAXM + 1) * MAXM];
    double e[2 * (MAXM + 1)];
    double y[2 * MAXM];
    double scale[MAXM + 1];
};

template <int TB>
__device__ __forceinline__ double blk_sum1(double v, TailLds& S) {
    constexpr int TW = TB / 64;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    v = wave_sum(v);
    if (lane == 0) S.red[wave] = v;
    __syncthreads();
    double s = 0.0;
#pragma unroll
    for (int wv = 0; wv < TW; ++wv) s += S.red[wv];
    __syncthreads();
    return s;
}

// One small ADR level for the single-workgroup GMRES.  The Krylov basis V_0..V_m is
// one contiguous allocation, V_q = V + q * n * n.
template <typename T>
struct BlockLevel {
    AdrGeom A;
    const T* px;
    const T* py;
    const cplx<T>* c0;
    const cplx<T>* b;
    cplx<T>* x;
    cplx<T>* V;
    int m;
};

template <typename T>
__device__ __forceinline__ BlockLevel<T> bsh_one(size_t o, BlockLevel<T> t) {
    t.px = bsh_one(o, t.px);
    t.py = bsh_one(o, t.py);
    t.c0 = bsh_one(o, t.c0);
    t.b = bsh_one(o, t.b);
    t.x = bsh_one(o, t.x);
    t.V = bsh_one(o, t.V);
    return t;
}

// GMRES(m) for the ADR operator of one small level (n*n <= NMAX) in one workgroup:
// x = x0 + argmin over K_m(M, r0) of ||b - M x||, x0 = 0 when x0_zero, m <= NQ.
// Arnoldi with two-pass classical Gram-Schmidt.  The current Arnoldi vector lives
// in LDS; each pass loads all basis values of a node at once and keeps one
// accumulator per basis vector, so the passes are not serialised over the basis.
// Stops early when h(j+1,j) <= tol beta.
template <typename T, int TB, int NQ, int NMAX>
__global__ __launch_bounds__(TB) void k_gmres_block(BlockLevel<T> L, int x0_zero, double tol, BatchIdx bi) {
    bshift(bi.off(), L);
    __shared__ TailLds S;
    __shared__ cplx<T> wl[NMAX];
    using C = cplx<T>;
    constexpr int TW = TB / 64;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int n = L.A.nx, N = L.A.nx * L.A.ny, m = L.m;  // n: nodes per row
    const C* V0 = x0_zero ? L.b : L.V;
    auto vget = [&](int q, int p) -> C { return q == 0 ? V0[p] : L.V[(size_t)q * N + p]; };
    // r0 and beta
    double nrm = 0.0;
    for (int p = tid; p < N; p += TB) {
        const int i = p / n, j = p - i * n;
        C v{};
        if (i > 0 && j > 0) v = x0_zero ? L.b[p] : adr_resid_at(L.A, L.px, L.py, L.c0, L.b, L.x, i, j);
        if (!x0_zero) L.V[p] = v;
        nrm += double(v.re) * double(v.re) + double(v.im) * double(v.im);
    }
    const double beta = sqrt(blk_sum1<TB>(nrm, S));
    if (!(beta > 0.0) || !isfinite(beta)) {
        if (x0_zero)
            for (int p = tid; p < N; p += TB) L.x[p] = C{};
        return;
    }
    if (tid == 0) S.scale[0] = 1.0 / beta;
    __syncthreads();
    int cols = m;
    for (int jj = 0; jj < m; ++jj) {
        const T sj = T(S.scale[jj]);
        const C* Vj = jj == 0 ? V0 : L.V + (size_t)jj * N;
        for (int p = tid; p < N; p += TB) {
            const int i = p / n, j = p - i * n;
            C v{};
            if (i > 0 && j > 0) v = sj * applyM_at(L.A, L.px, L.py, L.c0, Vj, i, j);
            wl[p] = v;
        }
        // pass 0: products; pass 1: subtract round-1 projection, products; pass 2: subtract, norm
        for (int pass = 0; pass < 3; ++pass) {
            double acc[2 * NQ];
#pragma unroll
            for (int q = 0; q < 2 * NQ; ++q) acc[q] = 0.0;
            double nn = 0.0;
            C cq[NQ];
#pragma unroll
            for (int q = 0; q < NQ; ++q) cq[q] = pass > 0 ? mk<T>(T(S.cq[2 * q]), T(S.cq[2 * q + 1])) : C{};
            for (int p = tid; p < N; p += TB) {
                C v[NQ];
#pragma unroll
                for (int q = 0; q < NQ; ++q) v[q] = q <= jj ? vget(q, p) : C{};
                C w = wl[p];
                if (pass > 0) {
#pragma unroll
                    for (int q = 0; q < NQ; ++q)
                        if (q <= jj) w = w - cq[q] * v[q];
                    wl[p] = w;
                }
                if (pass < 2) {
#pragma unroll
                    for (int q = 0; q < NQ; ++q) {
                        if (q <= jj) {
                            acc[2 * q] += double(v[q].re) * double(w.re) + double(v[q].im) * double(w.im);
                            acc[2 * q + 1] += double(v[q].re) * double(w.im) - double(v[q].im) * double(w.re);
                        }
                    }
                } else {
                    nn += double(w.re) * double(w.re) + double(w.im) * double(w.im);
                }
            }
            if (pass == 2) {
                const double hn = sqrt(blk_sum1<TB>(nn, S));
                if (tid == 0) {
                    S.H[2 * (jj + 1 + jj * (MAXM + 1))] = hn;
                    S.H[2 * (jj + 1 + jj * (MAXM + 1)) + 1] = 0.0;
                    S.scale[jj + 1] = hn > 0.0 ? 1.0 / hn : 0.0;
                }
                if (!isfinite(hn) || hn <= tol * beta) cols = jj + 1;
                break;
            }
#pragma unroll
            for (int q = 0; q < NQ; ++q) {
                if (q <= jj) {
                    const double ar = wave_sum(acc[2 * q]), ai = wave_sum(acc[2 * q + 1]);
                    if (lane == 0) {
                        S.red[wave * 2 * (MAXM + 1) + 2 * q] = ar;
                        S.red[wave * 2 * (MAXM + 1) + 2 * q + 1] = ai;
                    }
                }
            }
            __syncthreads();
            if (tid < 2 * (jj + 1)) {
                double sum = 0.0;
#pragma unroll
                for (int wv = 0; wv < TW; ++wv) sum += S.red[wv * 2 * (MAXM + 1) + tid];
                const double s = S.scale[tid >> 1];
                const double h = sum * s;  // <v_q, w>
                double* hp = S.H + 2 * ((tid >> 1) + jj * (MAXM + 1)) + (tid & 1);
                *hp = (pass ? *hp : 0.0) + h;
                S.cq[tid] = h * s;  // coefficient of V_q
            }
            __syncthreads();
        }
        if (cols == jj + 1) {
            __syncthreads();
            break;
        }
        if (jj + 1 < m) {
            C* W = L.V + (size_t)(jj + 1) * N;
            for (int p = tid; p < N; p += TB) W[p] = wl[p];
        }
        __syncthreads();
    }
    if (tid == 0) tail_lsq(S.H, beta, cols, S.y, S.e);
    __syncthreads();
    C cy[NQ];
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
        const double s = q < cols ? S.scale[q] : 0.0;
        cy[q] = mk<T>(T(S.y[2 * q] * s), T(S.y[2 * q + 1] * s));
    }
    for (int p = tid; p < N; p += TB) {
        C v = x0_zero ? C{} : L.x[p];
#pragma unroll
        for (int q = 0; q < NQ; ++q)
            if (q < cols) v = v + cy[q] * vget(q, p);
        L.x[p] = v;
    }
}

}  // namespace helm
