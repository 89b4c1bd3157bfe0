// GMRES(m) smoother for the ADR operator in s-step form (m <= 4).
//
// GMRES(m) from x0 returns x = x0 + z, z in span{r0, M r0, ..., M^{m-1} r0}, that
// minimises ||r0 - M z||.  With K_j = M^j r0 this is the least-squares problem
// min_c || K_0 - sum_{j=1..m} c_j K_j ||, and then x = x0 + sum_j c_j K_{j-1}.
// The Krylov vectors are never stored: each pass rebuilds them on a 64 x 16 tile
// plus a halo of one node per operator application, staged through LDS.
//   pass 1 (k_sstep_gram):    K_0..K_m on the tile, Gram matrix G = K^H K (FP64)
//   reduce (k_sstep_reduce):  the Gram partials summed, one block per entry
//   (the normalised Cholesky solve for c runs at the start of every combine block)
//   pass 2 (k_sstep_combine): K_0..K_{m-1} again, x_out = x0 + sum c_j K_{j-1}
// The normalised monomial basis of the ADR operator is well conditioned for
// m <= 4 (condition numbers of 5-40 measured on the workloads), so the normal
// equations lose at most about three digits of FP64 accuracy.
#pragma once

#include "kernels_krylov.hpp"

namespace helm {

template <int M, bool X0>
struct SStep {
    static constexpr int HMAX = M + (X0 ? 1 : 0);  // halo of the first loaded field
    static constexpr int PW = TX + 2 * HMAX;
    static constexpr int PH = TY + 2 * HMAX;
    static constexpr int PN = PW * PH;
    static constexpr int NG = (M + 1) * (M + 1);  // doubles of the Gram (diag real + upper complex)
};

// Top-left node of tile t.
__device__ __forceinline__ void sstep_tile(int n, int t, int& j0, int& i0) {
    const int ntx = (n + TX - 1) / TX;
    j0 = (t % ntx) * TX;
    i0 = (t / ntx) * TY;
}

// M applied at LDS position (li, lj) of a field stored with padded width PW.
template <typename T, int PW>
__device__ __forceinline__ cplx<T> applyM_lds(const AdrGeom& A, const cplx<T>* __restrict__ s, int li, int lj, T fx,
                                              T fy, cplx<T> cc) {
    const cplx<T> c = s[li * PW + lj];
    const cplx<T> w = s[li * PW + lj - 1], e = s[li * PW + lj + 1];
    const cplx<T> so = s[(li - 1) * PW + lj], nn = s[(li + 1) * PW + lj];
    const T ax = fx < T(0) ? -fx : fx, ay = fy < T(0) ? -fy : fy;
    const cplx<T> lap = T(A.inv_h2) * (T(4) * c - (((so + nn) + w) + e));
    const cplx<T> U = T(A.inv_2h) * (((((T(2) * (ax + ay)) * c - (fx + ax) * w) + (fx - ax) * e) - (fy + ay) * so) +
                                    (fy - ay) * nn);
    const cplx<T> adv = mk<T>(T(A.two_sk) * U.im, -T(A.two_sk) * U.re);
    return lap + (adv + cc * c);
}

// dst = M src on the tile region with halo h (src valid on halo h+1); zero off the unknowns.
template <typename T, int M, bool X0>
__device__ __forceinline__ void sstep_stage(const AdrGeom& A, const T* __restrict__ px, const T* __restrict__ py,
                                            const cplx<T>* __restrict__ c0, const cplx<T>* __restrict__ src,
                                            cplx<T>* __restrict__ dst, int h, int i0, int j0) {
    using S = SStep<M, X0>;
    const int tid = threadIdx.x + threadIdx.y * TX;
    const int rw = TX + 2 * h, rh = TY + 2 * h;
    const int off = S::HMAX - h;
    for (int q = tid; q < rw * rh; q += BLOCK) {
        const int ri = q / rw, rj = q - ri * rw;
        const int gi = i0 - h + ri, gj = j0 - h + rj;
        const int li = off + ri, lj = off + rj;
        cplx<T> v{};
        if (gi >= 1 && gj >= 1 && gi < A.n && gj < A.n) {
            const size_t p = (size_t)gi * A.n + gj;
            v = applyM_lds<T, S::PW>(A, src, li, lj, px[p], py[p], c0[p]);
        }
        dst[li * S::PW + lj] = v;
    }
    __syncthreads();
}

// Loads K_0 = b - M x0 (X0) or K_0 = b on the region with halo M (+0), into buffer k0.
template <typename T, int M, bool X0>
__device__ __forceinline__ void sstep_load(const AdrGeom& A, const T* __restrict__ px, const T* __restrict__ py,
                                           const cplx<T>* __restrict__ c0, const cplx<T>* __restrict__ b,
                                           const cplx<T>* __restrict__ x0, cplx<T>* __restrict__ xs,
                                           cplx<T>* __restrict__ k0, int hk0, int i0, int j0) {
    using S = SStep<M, X0>;
    const int tid = threadIdx.x + threadIdx.y * TX;
    if (X0) {
        const int h = hk0 + 1;
        const int rw = TX + 2 * h, rh = TY + 2 * h;
        const int off = S::HMAX - h;
        for (int q = tid; q < rw * rh; q += BLOCK) {
            const int ri = q / rw, rj = q - ri * rw;
            const int gi = i0 - h + ri, gj = j0 - h + rj;
            cplx<T> v{};
            if (gi >= 1 && gj >= 1 && gi < A.n && gj < A.n) v = x0[(size_t)gi * A.n + gj];
            xs[(off + ri) * S::PW + off + rj] = v;
        }
        __syncthreads();
    }
    const int h = hk0;
    const int rw = TX + 2 * h, rh = TY + 2 * h;
    const int off = S::HMAX - h;
    for (int q = tid; q < rw * rh; q += BLOCK) {
        const int ri = q / rw, rj = q - ri * rw;
        const int gi = i0 - h + ri, gj = j0 - h + rj;
        const int li = off + ri, lj = off + rj;
        cplx<T> v{};
        if (gi >= 1 && gj >= 1 && gi < A.n && gj < A.n) {
            const size_t p = (size_t)gi * A.n + gj;
            v = b[p];
            if (X0) v = v - applyM_lds<T, S::PW>(A, xs, li, lj, px[p], py[p], c0[p]);
        }
        k0[li * S::PW + lj] = v;
    }
    __syncthreads();
}

// Interior points of a tile per thread, and the interior values of a buffer copied
// to registers (point q = tid + e * BLOCK of the tile).
constexpr int IPT = TX * TY / BLOCK;

template <typename T, int PW, int HMAX>
__device__ __forceinline__ void sstep_keep(const cplx<T>* __restrict__ buf, cplx<T> (&k)[IPT], int tid) {
#pragma unroll
    for (int e = 0; e < IPT; ++e) {
        const int q = tid + e * BLOCK;
        const int ri = q / TX, rj = q - ri * TX;
        k[e] = buf[(HMAX + ri) * PW + HMAX + rj];
    }
}

// Pass 1: K_0..K_M on the tile and the Gram matrix; per-block sums to partials[blk * NG].
// Layout of the NG doubles: G(i,i) real for i = 0..M, then G(i,j), i < j, as (re, im).
// Two LDS buffers alternate between the stages; the interior values of every K_j
// are kept in registers as soon as the stage has produced them.
template <typename T, int M, bool X0>
__global__ __launch_bounds__(BLOCK) void k_sstep_gram(AdrGeom A, const T* __restrict__ px, const T* __restrict__ py,
                                                      const cplx<T>* __restrict__ c0, const cplx<T>* __restrict__ b,
                                                      const cplx<T>* __restrict__ x0, double* __restrict__ partials) {
    using S = SStep<M, X0>;
    __shared__ cplx<T> bufA[S::PN], bufB[S::PN];
    __shared__ double red[4 * S::NG];
    __shared__ double sums[S::NG];
    // FP64 products: the unscaled powers M^j K_0 span many decades (|M| ~ 8/h^2)
    double acc[S::NG];
#pragma unroll
    for (int q = 0; q < S::NG; ++q) acc[q] = 0.0;
    const int tid = threadIdx.x + threadIdx.y * TX;
    int t0, t1;
    tile_chunk(A.n, t0, t1);
    for (int t = t0; t < t1; ++t) {
        int j0, i0;
        sstep_tile(A.n, t, j0, i0);
        __syncthreads();
        // x0 staging in bufB, K_0 in bufA, then K_j alternating
        sstep_load<T, M, X0>(A, px, py, c0, b, x0, bufB, bufA, M, i0, j0);
        cplx<T> k[M + 1][IPT];
        sstep_keep<T, S::PW, S::HMAX>(bufA, k[0], tid);
        cplx<T>* src = bufA;
        cplx<T>* dst = bufB;
#pragma unroll
        for (int j = 1; j < M; ++j) {
            sstep_stage<T, M, X0>(A, px, py, c0, src, dst, M - j, i0, j0);
            sstep_keep<T, S::PW, S::HMAX>(dst, k[j], tid);
            cplx<T>* tmp = src;
            src = dst;
            dst = tmp;
        }
#pragma unroll
        for (int e = 0; e < IPT; ++e) {
            const int q = tid + e * BLOCK;
            const int ri = q / TX, rj = q - ri * TX;
            const int gi = i0 + ri, gj = j0 + rj;
            if (gi < 1 || gj < 1 || gi >= A.n || gj >= A.n) continue;
            const int li = S::HMAX + ri, lj = S::HMAX + rj;
            const size_t p = (size_t)gi * A.n + gj;
            k[M][e] = applyM_lds<T, S::PW>(A, src, li, lj, px[p], py[p], c0[p]);
            int o = M + 1;
#pragma unroll
            for (int i = 0; i <= M; ++i) {
                const double ar = double(k[i][e].re), ai = double(k[i][e].im);
                acc[i] += ar * ar + ai * ai;
#pragma unroll
                for (int jv = i + 1; jv <= M; ++jv) {
                    const double br = double(k[jv][e].re), bi = double(k[jv][e].im);
                    acc[o] += ar * br + ai * bi;
                    acc[o + 1] += ar * bi - ai * br;
                    o += 2;
                }
            }
        }
    }
    block_sum<S::NG, 4>(acc, S::NG, red, sums);
    store_partials(sums, S::NG, partials);
}

// Normalised Cholesky solve of the normal equations from the Gram sums (layout of
// k_sstep_gram); one thread.  yr, yi: coefficients c_j of K_{j-1}; cols: columns kept
// (columns after the first negligible pivot are dropped); beta = ||K_0||.
template <int M>
__device__ __forceinline__ void sstep_small_solve(const double* __restrict__ sums, double breakdown_tol,
                                                  double (&yr)[M], double (&yi)[M], int& cols, double& beta) {
    // Hermitian G(i,j), i,j = 0..M; every loop below has compile-time bounds so that
    // the small arrays stay in registers.
    double gr[M + 1][M + 1], gi[M + 1][M + 1];
#pragma unroll
    for (int i = 0; i <= M; ++i) {
        gr[i][i] = sums[i];
        gi[i][i] = 0.0;
    }
    {
        int o = M + 1;
#pragma unroll
        for (int i = 0; i <= M; ++i)
#pragma unroll
            for (int j = i + 1; j <= M; ++j) {
                gr[i][j] = sums[o];
                gi[i][j] = sums[o + 1];
                gr[j][i] = sums[o];
                gi[j][i] = -sums[o + 1];
                o += 2;
            }
    }
    beta = sqrt(gr[0][0]);
#pragma unroll
    for (int i = 0; i < M; ++i) yr[i] = yi[i] = 0.0;
    cols = 0;
    if (beta > 0.0 && isfinite(beta)) {
        double d[M + 1];
#pragma unroll
        for (int i = 0; i <= M; ++i) d[i] = sqrt(gr[i][i]);
        // normalised normal equations N c' = r, N(i,j) = G(i,j)/(d_i d_j), r(i) = G(i,0)/(d_i d_0)
        double Lr[M][M], Li[M][M];
#pragma unroll
        for (int i = 0; i < M; ++i)
#pragma unroll
            for (int j = 0; j < M; ++j) {
                const double s = (d[i + 1] > 0 && d[j + 1] > 0) ? 1.0 / (d[i + 1] * d[j + 1]) : 0.0;
                Lr[i][j] = gr[i + 1][j + 1] * s;
                Li[i][j] = gi[i + 1][j + 1] * s;
            }
        // Cholesky N = L L^H; columns after the first negligible pivot are dropped
        bool ok = true;
#pragma unroll
        for (int j = 0; j < M; ++j) {
            double p = Lr[j][j];
#pragma unroll
            for (int q = 0; q < j; ++q) p -= Lr[j][q] * Lr[j][q] + Li[j][q] * Li[j][q];
            ok = ok && (p > breakdown_tol * breakdown_tol);
            if (ok) cols = j + 1;
            const double lj = ok ? sqrt(p) : 1.0;
            Lr[j][j] = lj;
            Li[j][j] = 0.0;
#pragma unroll
            for (int i = j + 1; i < M; ++i) {
                double sr = Lr[i][j], si = Li[i][j];
#pragma unroll
                for (int q = 0; q < j; ++q) {
                    sr -= Lr[i][q] * Lr[j][q] + Li[i][q] * Li[j][q];
                    si -= Li[i][q] * Lr[j][q] - Lr[i][q] * Li[j][q];
                }
                Lr[i][j] = sr / lj;
                Li[i][j] = si / lj;
            }
        }
        double zr[M], zi[M];
#pragma unroll
        for (int i = 0; i < M; ++i) {  // L z = r  (rows >= cols give zero)
            const double s = 1.0 / (d[i + 1] * d[0]);
            double sr = gr[i + 1][0] * s, si = gi[i + 1][0] * s;
#pragma unroll
            for (int q = 0; q < i; ++q) {
                sr -= Lr[i][q] * zr[q] - Li[i][q] * zi[q];
                si -= Lr[i][q] * zi[q] + Li[i][q] * zr[q];
            }
            zr[i] = i < cols ? sr / Lr[i][i] : 0.0;
            zi[i] = i < cols ? si / Lr[i][i] : 0.0;
        }
#pragma unroll
        for (int i = M - 1; i >= 0; --i) {  // L^H c' = z
            double sr = zr[i], si = zi[i];
#pragma unroll
            for (int q = i + 1; q < M; ++q) {
                sr -= Lr[q][i] * zr[q] + Li[q][i] * zi[q];
                si -= Lr[q][i] * zi[q] - Li[q][i] * zr[q];
            }
            zr[i] = i < cols ? sr / Lr[i][i] : 0.0;
            zi[i] = i < cols ? si / Lr[i][i] : 0.0;
        }
#pragma unroll
        for (int i = 0; i < M; ++i) {  // c_j = c'_j d_0 / d_j
            const double s = i < cols ? d[0] / d[i + 1] : 0.0;
            yr[i] = zr[i] * s;
            yi[i] = zi[i] * s;
        }
    }
}

// Grid reduction of the Gram partials: block v sums partials[v * nblk + b] over b
// (fixed order) into gsum[v]; NG blocks of BLOCK threads.
__global__ __launch_bounds__(BLOCK) void k_sstep_reduce(const double* __restrict__ partials, int nblk,
                                                        double* __restrict__ gsum) {
    __shared__ double red[4];
    __shared__ double sums[1];
    const int v = blockIdx.x;
    double acc[1] = {0.0};
    for (int b = threadIdx.x; b < nblk; b += BLOCK) acc[0] += partials[(size_t)v * nblk + b];
    block_sum<1, 4>(acc, 1, red, sums);
    if (threadIdx.x == 0) gsum[v] = sums[0];
}

// Pass 2: x_out = x0 + sum_{j=1..cols} c_j K_{j-1} on the tile interior, with the
// coefficients solved per block from the Gram sums gsum (thread 0, overlapped with
// the other threads' tile loads); block 0 also records them in K.
template <typename T, int M, bool X0>
__global__ __launch_bounds__(BLOCK) void k_sstep_combine(AdrGeom A, const T* __restrict__ px, const T* __restrict__ py,
                                                         const cplx<T>* __restrict__ c0, const cplx<T>* __restrict__ b,
                                                         const cplx<T>* __restrict__ x0,
                                                         const double* __restrict__ gsum, double breakdown_tol,
                                                         KrylovScal* K, cplx<T>* __restrict__ xout) {
    using S = SStep<M, X0>;
    __shared__ cplx<T> bufA[S::PN], bufB[S::PN];
    __shared__ cplx<T> cs[M];
    int j0, i0;
    {
        int jj, ii;
        tile_origin(A.n, jj, ii);
        j0 = jj - (int)threadIdx.x;
        i0 = ii - (int)threadIdx.y * RPT;
    }
    const int tid = threadIdx.x + threadIdx.y * TX;
    if (tid == 0) {
        double yr[M], yi[M], beta;
        int cols;
        sstep_small_solve<M>(gsum, breakdown_tol, yr, yi, cols, beta);
#pragma unroll
        for (int j = 0; j < M; ++j) cs[j] = mk<T>(T(yr[j]), T(yi[j]));
        if (blockIdx.x == 0) {
            K->beta = beta;
#pragma unroll
            for (int j = 0; j < M; ++j) {
                K->y[2 * j] = yr[j];
                K->y[2 * j + 1] = yi[j];
            }
            K->cols = cols;
            K->done = isfinite(beta) ? 1 : 2;
        }
    }
    // K_0 needs halo M-1 here (the loads end with a barrier, which also publishes cs)
    sstep_load<T, M, X0>(A, px, py, c0, b, x0, bufB, bufA, M - 1, i0, j0);
    cplx<T> k[M][IPT];
    sstep_keep<T, S::PW, S::HMAX>(bufA, k[0], tid);
    cplx<T>* src = bufA;
    cplx<T>* dst = bufB;
#pragma unroll
    for (int j = 1; j < M; ++j) {
        sstep_stage<T, M, X0>(A, px, py, c0, src, dst, M - 1 - j, i0, j0);
        sstep_keep<T, S::PW, S::HMAX>(dst, k[j], tid);
        cplx<T>* tmp = src;
        src = dst;
        dst = tmp;
    }
    cplx<T> c[M];
#pragma unroll
    for (int j = 0; j < M; ++j) c[j] = cs[j];
#pragma unroll
    for (int e = 0; e < IPT; ++e) {
        const int q = tid + e * BLOCK;
        const int ri = q / TX, rj = q - ri * TX;
        const int gi = i0 + ri, gj = j0 + rj;
        if (gi >= A.n || gj >= A.n) continue;
        const size_t p = (size_t)gi * A.n + gj;
        cplx<T> v{};
        if (gi >= 1 && gj >= 1) {
            v = X0 ? x0[p] : cplx<T>{};
#pragma unroll
            for (int j = 0; j < M; ++j) v = v + c[j] * k[j][e];
        }
        xout[p] = v;
    }
}

}  // namespace helm
