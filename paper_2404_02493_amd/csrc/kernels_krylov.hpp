// Krylov kernels shared by the GMRES(m) ADR smoother and the outer FGMRES:
// fused operator + inner-product passes, two-pass classical Gram-Schmidt with
// re-orthogonalisation, the device-side Hessenberg least squares, and the
// final combination x = x0 + V y.  All inner products accumulate in FP64 and
// every grid reduction ends in the last block (no host round trip).
#pragma once

#include "kernels_adr.hpp"

namespace helm {

template <typename T>
struct VecSet {
    const cplx<T>* v[MAXM + 1];
};

__device__ __forceinline__ double* Hp(KrylovScal* K, int i, int j) { return K->H + 2 * (i + j * (MAXM + 1)); }

// Solve min || beta e1 - H y || for the leading (cols+1) x cols block with complex
// Givens rotations (one thread; works in K->R / K->e, global memory).
__device__ inline void ks_least_squares(KrylovScal* K, int cols) {
    double* R = K->R;
    double* e = K->e;
    auto Rp = [&](int i, int j) { return R + 2 * (i + j * (MAXM + 1)); };
    for (int j = 0; j < cols; ++j)
        for (int i = 0; i <= j + 1; ++i) {
            Rp(i, j)[0] = Hp(K, i, j)[0];
            Rp(i, j)[1] = Hp(K, i, j)[1];
        }
    for (int i = 0; i <= cols; ++i) e[2 * i] = e[2 * i + 1] = 0.0;
    e[0] = K->beta;
    for (int j = 0; j < cols; ++j) {
        // rotation j acts on rows j, j+1; rows j..j+1 of columns < j are already zero
        double ar = Rp(j, j)[0], ai = Rp(j, j)[1];
        double br = Rp(j + 1, j)[0], bi = Rp(j + 1, j)[1];
        double na = hypot(ar, ai), nb = hypot(br, bi);
        double c, sr, si;  // [c s; -conj(s) c], s = (a/|a|) conj(b) / rho
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
            double xr = Rp(j, q)[0], xi = Rp(j, q)[1];
            double yr = Rp(j + 1, q)[0], yi = Rp(j + 1, q)[1];
            Rp(j, q)[0] = c * xr + (sr * yr - si * yi);
            Rp(j, q)[1] = c * xi + (sr * yi + si * yr);
            Rp(j + 1, q)[0] = -(sr * xr + si * xi) + c * yr;
            Rp(j + 1, q)[1] = -(sr * xi - si * xr) + c * yi;
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
            double hr_ = Rp(i, q)[0], hi_ = Rp(i, q)[1];
            double yr = K->y[2 * q], yi = K->y[2 * q + 1];
            accr -= hr_ * yr - hi_ * yi;
            acci -= hr_ * yi + hi_ * yr;
        }
        double dr = Rp(i, i)[0], di = Rp(i, i)[1];
        double d = dr * dr + di * di;
        K->y[2 * i] = (accr * dr + acci * di) / d;
        K->y[2 * i + 1] = (acci * dr - accr * di) / d;
    }
    for (int i = cols; i < MAXM; ++i) K->y[2 * i] = K->y[2 * i + 1] = 0.0;
}

// Partial ||x||^2 of a Krylov start vector (finalize with FIN_INIT).
template <typename T>
__global__ __launch_bounds__(BLOCK) void k_krylov_init_norm(size_t N, const cplx<T>* __restrict__ x, double* partials) {
    __shared__ double red[4];
    __shared__ double sums[1];
    double acc[1] = {0.0};
    for (size_t p = blockIdx.x * (size_t)BLOCK + threadIdx.x; p < N; p += (size_t)gridDim.x * BLOCK) {
        cplx<T> v = x[p];
        acc[0] += double(v.re) * double(v.re) + double(v.im) * double(v.im);
    }
    block_sum<1, 4>(acc, 1, red, sums);
    store_partials(sums, 1, partials);
}

// r0 = b - M x (ADR operator) written to r0, partial ||r0||^2 (finalize with FIN_INIT).
template <typename T>
__global__ __launch_bounds__(BLOCK) void k_adr_residual_init(AdrGeom A, const T* __restrict__ px, const T* __restrict__ py,
                                                             const cplx<T>* __restrict__ c0, const cplx<T>* __restrict__ b,
                                                             const cplx<T>* __restrict__ x, cplx<T>* __restrict__ r0,
                                                             double* partials) {
    __shared__ double red[4];
    __shared__ double sums[1];
    double acc[1] = {0.0};
    int t0, t1;
    tile_chunk(A.n, t0, t1);
    for (int t = t0; t < t1; ++t) {
        int j, i0;
        tile_xy(A.n, t, j, i0);
        if (j >= A.n) continue;
        for (int r = 0; r < RPT; ++r) {
            const int i = i0 + r;
            if (i >= A.n) break;
            cplx<T> v{};
            if (i > 0 && j > 0) v = adr_resid_at(A, px, py, c0, b, x, i, j);
            r0[(size_t)i * A.n + j] = v;
            acc[0] += double(v.re) * double(v.re) + double(v.im) * double(v.im);
        }
    }
    block_sum<1, 4>(acc, 1, red, sums);
    store_partials(sums, 1, partials);
}

// Accumulates sum conj(V_i) * w over i <= jj into acc (unscaled).  Per-thread partial
// sums run in the working precision A (a thread sums a few dozen products); the
// block and grid reductions are FP64.
template <typename T, int NV, typename A = double>
__device__ __forceinline__ void acc_dots(A (&acc)[2 * NV + 2], const VecSet<T>& V, int jj, size_t p, cplx<T> w) {
#pragma unroll
    for (int i = 0; i < NV; ++i) {
        if (i <= jj) {
            cplx<T> v = V.v[i][p];
            acc[2 * i] += A(v.re) * A(w.re) + A(v.im) * A(w.im);
            acc[2 * i + 1] += A(v.re) * A(w.im) - A(v.im) * A(w.re);
        }
    }
}

template <int K, typename A>
__device__ __forceinline__ void to_double(const A (&a)[K], double (&d)[K]) {
#pragma unroll
    for (int q = 0; q < K; ++q) d[q] = double(a[q]);
}

// Arnoldi matvec pass with the ADR operator: w = M (scale[jj] V_jj); partial sums of
// conj(V_i) w, i <= jj (finalize with FIN_MV).
template <typename T, int NV>
__global__ __launch_bounds__(BLOCK) void k_arnoldi_adr(AdrGeom A, const T* __restrict__ px, const T* __restrict__ py,
                                                       const cplx<T>* __restrict__ c0, VecSet<T> V, int jj,
                                                       cplx<T>* __restrict__ w, const KrylovScal* K, double* partials) {
    __shared__ double red[4 * (2 * NV + 2)];
    __shared__ double sums[2 * NV + 2];
    if (K->done) return;
    const T sj = T(K->scale[jj]);
    double acc[2 * NV + 2];
#pragma unroll
    for (int q = 0; q < 2 * NV + 2; ++q) acc[q] = 0.0;
    int t0, t1;
    tile_chunk(A.n, t0, t1);
    for (int t = t0; t < t1; ++t) {
        int j, i0;
        tile_xy(A.n, t, j, i0);
        if (j >= A.n) continue;
        for (int r = 0; r < RPT; ++r) {
            const int i = i0 + r;
            if (i >= A.n) break;
            const size_t p = (size_t)i * A.n + j;
            cplx<T> v{};
            if (i > 0 && j > 0) v = sj * applyM_at(A, px, py, c0, V.v[jj], i, j);
            w[p] = v;
            acc_dots<T, NV>(acc, V, jj, p, v);
        }
    }
    block_sum<2 * NV + 2, 4>(acc, 2 * (jj + 1), red, sums);
    store_partials(sums, 2 * (jj + 1), partials);
}

// Arnoldi matvec pass with the Helmholtz operator on z: w = A (s z), s = scale[jj] if
// use_scale else 1; partial sums of conj(V_i) w  (FGMRES: z = C(0, V_jj) or C(0, v_jj)).
template <typename T, int NV>
__global__ __launch_bounds__(BLOCK) void k_arnoldi_helm(Geom G, const T* __restrict__ n2, const cplx<T>* __restrict__ z,
                                                        int use_scale, VecSet<T> V, int jj, cplx<T>* __restrict__ w,
                                                        const KrylovScal* K, double* partials) {
    __shared__ double red[4 * (2 * NV + 2)];
    __shared__ double sums[2 * NV + 2];
    if (K->done) return;
    const T sj = use_scale ? T(K->scale[jj]) : T(1);
    T acc[2 * NV + 2];
#pragma unroll
    for (int q = 0; q < 2 * NV + 2; ++q) acc[q] = T(0);
    int t0, t1;
    tile_chunk(G.n, t0, t1);
    for (int t = t0; t < t1; ++t) {
        int j, i0;
        tile_xy(G.n, t, j, i0);
        if (j >= G.n) continue;
        for (int r = 0; r < RPT; ++r) {
            const int i = i0 + r;
            if (i >= G.n) break;
            const size_t p = (size_t)i * G.n + j;
            cplx<T> v{};
            if (i > 0 && j > 0) v = sj * applyA_at(G, n2, z, i, j, false);
            w[p] = v;
            acc_dots<T, NV, T>(acc, V, jj, p, v);
        }
    }
    double accd[2 * NV + 2];
    to_double(acc, accd);
    block_sum<2 * NV + 2, 4>(accd, 2 * (jj + 1), red, sums);
    store_partials(sums, 2 * (jj + 1), partials);
}

// Loads the coefficients c_i = dots_i * scale_i (complex) of the current correction.
template <typename T, int NV>
__device__ __forceinline__ void load_coefs(const KrylovScal* K, int jj, cplx<T> (&c)[NV]) {
#pragma unroll
    for (int i = 0; i < NV; ++i) {
        if (i <= jj) {
            double s = K->scale[i];
            c[i] = mk<T>(T(K->dots[2 * i] * s), T(K->dots[2 * i + 1] * s));
        } else {
            c[i] = cplx<T>{};
        }
    }
}

// Gram-Schmidt pass 1: w -= sum_i dots_i v_i, partial sums of conj(V_i) w (FIN_ORTH1).
template <typename T, int NV>
__global__ __launch_bounds__(BLOCK) void k_orth_pass1(size_t N, VecSet<T> V, int jj, cplx<T>* __restrict__ w,
                                                      const KrylovScal* K, double* partials) {
    __shared__ double red[4 * (2 * NV + 2)];
    __shared__ double sums[2 * NV + 2];
    __shared__ cplx<T> c[NV];
    if (K->done) return;
    if ((int)threadIdx.x < NV) {
        const int i = threadIdx.x;
        c[i] = i <= jj ? mk<T>(T(K->dots[2 * i] * K->scale[i]), T(K->dots[2 * i + 1] * K->scale[i])) : cplx<T>{};
    }
    __syncthreads();
    T acc[2 * NV + 2];
#pragma unroll
    for (int q = 0; q < 2 * NV + 2; ++q) acc[q] = T(0);
    for (size_t p = blockIdx.x * (size_t)BLOCK + threadIdx.x; p < N; p += (size_t)gridDim.x * BLOCK) {
        cplx<T> x = w[p];
#pragma unroll
        for (int i = 0; i < NV; ++i)
            if (i <= jj) x = x - c[i] * V.v[i][p];
        w[p] = x;
        acc_dots<T, NV, T>(acc, V, jj, p, x);
    }
    double accd[2 * NV + 2];
    to_double(acc, accd);
    block_sum<2 * NV + 2, 4>(accd, 2 * (jj + 1), red, sums);
    store_partials(sums, 2 * (jj + 1), partials);
}

// Gram-Schmidt pass 2: w -= sum_i dots2_i v_i, partial ||w||^2 (FIN_ORTH2).
template <typename T, int NV>
__global__ __launch_bounds__(BLOCK) void k_orth_pass2(size_t N, VecSet<T> V, int jj, cplx<T>* __restrict__ w,
                                                      const KrylovScal* K, double* partials) {
    __shared__ double red[4];
    __shared__ double sums[1];
    if (K->done) return;
    cplx<T> c[NV];
    load_coefs<T, NV>(K, jj, c);
    double acc[1] = {0.0};
    for (size_t p = blockIdx.x * (size_t)BLOCK + threadIdx.x; p < N; p += (size_t)gridDim.x * BLOCK) {
        cplx<T> x = w[p];
#pragma unroll
        for (int i = 0; i < NV; ++i)
            if (i <= jj) x = x - c[i] * V.v[i][p];
        w[p] = x;
        acc[0] += double(x.re) * double(x.re) + double(x.im) * double(x.im);
    }
    block_sum<1, 4>(acc, 1, red, sums);
    store_partials(sums, 1, partials);
}

// ---- wave-split passes for the outer FGMRES (up to MAXM + 1 basis vectors)
// The 4 wavefronts of a block walk the same elements, 64 * E at a time; wave w owns
// the basis vectors i = w, w + 4, ...: it loads them once per element, adds its
// share of the projection (exchanged through LDS) and accumulates their inner
// products with the updated vector.  Each vector is read once per pass and a thread
// holds the accumulators of a quarter of the basis only.
constexpr int WS_WAVES = 4;

template <typename T>
struct WsShape {
    static constexpr int E = sizeof(T) == 4 ? 4 : 2;  // elements per lane per step
    static constexpr int STEP = 64 * E;
};

// Contiguous element range of this block, a multiple of the step.
template <typename T>
__device__ __forceinline__ void ws_range(size_t N, size_t& b0, size_t& b1) {
    const size_t step = WsShape<T>::STEP;
    const size_t per = ((N + gridDim.x - 1) / gridDim.x + step - 1) / step * step;
    b0 = (size_t)blockIdx.x * per;
    b1 = b0 + per < N ? b0 + per : N;
}

// Per-wave accumulators (vectors i = wave + 4k) -> partials[(2i + c) * nblk + block].
template <typename T, int NPW>
__device__ __forceinline__ void ws_store(const T (&acc)[2 * NPW], int jj, double* sums, double* partials) {
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
#pragma unroll
    for (int k = 0; k < NPW; ++k) {
        const int i = wave + WS_WAVES * k;
        if (i <= jj) {
            const double re = wave_sum(double(acc[2 * k])), im = wave_sum(double(acc[2 * k + 1]));
            if (lane == 0) {
                sums[2 * i] = re;
                sums[2 * i + 1] = im;
            }
        }
    }
    __syncthreads();
    store_partials(sums, 2 * (jj + 1), partials);
}

// w = A (s z) on the fine grid and partial conj(V_i) w, i <= jj (finalize with FIN_MV).
// Wave e of the block evaluates the stencil for slice e of the step (E slices of 64
// elements, E = 4 waves for complex64) and shares it through LDS, so z is read once.
template <typename T, int NV>
__global__ __launch_bounds__(BLOCK) void k_arnoldi_helm_ws(Geom G, const T* __restrict__ n2,
                                                           const cplx<T>* __restrict__ z, int use_scale, VecSet<T> V,
                                                           int jj, cplx<T>* __restrict__ w, const KrylovScal* K,
                                                           double* partials) {
    constexpr int NPW = (NV + WS_WAVES - 1) / WS_WAVES;
    constexpr int E = WsShape<T>::E;
    __shared__ double sums[2 * NV + 2];
    __shared__ cplx<T> xs[E][64];
    if (K->done) return;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const T sj = use_scale ? T(K->scale[jj]) : T(1);
    const size_t N = (size_t)G.n * G.n;
    T acc[2 * NPW];
#pragma unroll
    for (int q = 0; q < 2 * NPW; ++q) acc[q] = T(0);
    size_t b0, b1;
    ws_range<T>(N, b0, b1);
    for (size_t base = b0; base < b1; base += WsShape<T>::STEP) {
        // stencil slices: wave w computes slices w, w + 4, ... (E <= 4: one or none)
        for (int e = wave; e < E; e += WS_WAVES) {
            const size_t p = base + (size_t)e * 64 + lane;
            cplx<T> v{};
            if (p < b1) {
                const int i = (int)(p / G.n), j = (int)(p % G.n);
                if (i > 0 && j > 0) v = sj * applyA_at(G, n2, z, i, j, false);
                w[p] = v;
            }
            xs[e][lane] = v;
        }
        __syncthreads();
        cplx<T> x[E];
#pragma unroll
        for (int e = 0; e < E; ++e) x[e] = xs[e][lane];
#pragma unroll
        for (int k = 0; k < NPW; ++k) {
            const int iv = wave + WS_WAVES * k;
            if (iv <= jj) {
#pragma unroll
                for (int e = 0; e < E; ++e) {
                    const size_t p = base + (size_t)e * 64 + lane;
                    if (p < b1) {
                        const cplx<T> v = V.v[iv][p];
                        acc[2 * k] += v.re * x[e].re + v.im * x[e].im;
                        acc[2 * k + 1] += v.re * x[e].im - v.im * x[e].re;
                    }
                }
            }
        }
        __syncthreads();
    }
    ws_store<T, NPW>(acc, jj, sums, partials);
}

// Gram-Schmidt pass 1: w -= sum_i dots_i v_i; partial conj(V_i) w (FIN_ORTH1).
template <typename T, int NV>
__global__ __launch_bounds__(BLOCK) void k_orth_pass1_ws(size_t N, VecSet<T> V, int jj, cplx<T>* __restrict__ w,
                                                         const KrylovScal* K, double* partials) {
    constexpr int NPW = (NV + WS_WAVES - 1) / WS_WAVES;
    constexpr int E = WsShape<T>::E;
    __shared__ cplx<T> cs[NV];
    __shared__ cplx<T> part[WS_WAVES][E][64];
    __shared__ double sums[2 * NV + 2];
    if (K->done) return;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    if ((int)threadIdx.x < NV) {
        const int i = threadIdx.x;
        cs[i] = i <= jj ? mk<T>(T(K->dots[2 * i] * K->scale[i]), T(K->dots[2 * i + 1] * K->scale[i])) : cplx<T>{};
    }
    __syncthreads();
    T acc[2 * NPW];
#pragma unroll
    for (int q = 0; q < 2 * NPW; ++q) acc[q] = T(0);
    size_t b0, b1;
    ws_range<T>(N, b0, b1);
    for (size_t base = b0; base < b1; base += WsShape<T>::STEP) {
        cplx<T> v[NPW][E];
        cplx<T> px[E], wv[E];
#pragma unroll
        for (int e = 0; e < E; ++e) {
            // every wave reads w before the barrier; wave 0 overwrites it after
            const size_t p = base + (size_t)e * 64 + lane;
            px[e] = cplx<T>{};
            wv[e] = p < b1 ? w[p] : cplx<T>{};
        }
#pragma unroll
        for (int k = 0; k < NPW; ++k) {
            const int iv = wave + WS_WAVES * k;
#pragma unroll
            for (int e = 0; e < E; ++e) {
                const size_t p = base + (size_t)e * 64 + lane;
                v[k][e] = (iv <= jj && p < b1) ? V.v[iv][p] : cplx<T>{};
                px[e] = px[e] + cs[iv <= jj ? iv : 0] * v[k][e];
            }
        }
#pragma unroll
        for (int e = 0; e < E; ++e) part[wave][e][lane] = px[e];
        __syncthreads();
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const size_t p = base + (size_t)e * 64 + lane;
            cplx<T> x{};
            if (p < b1) {
                x = wv[e] - ((part[0][e][lane] + part[1][e][lane]) + (part[2][e][lane] + part[3][e][lane]));
                if (wave == 0) w[p] = x;
            }
#pragma unroll
            for (int k = 0; k < NPW; ++k) {
                acc[2 * k] += v[k][e].re * x.re + v[k][e].im * x.im;
                acc[2 * k + 1] += v[k][e].re * x.im - v[k][e].im * x.re;
            }
        }
        __syncthreads();
    }
    ws_store<T, NPW>(acc, jj, sums, partials);
}

enum FinOp { FIN_INIT = 0, FIN_MV = 1, FIN_ORTH1 = 2, FIN_ORTH2 = 3 };

// One block: sums the partials of the previous Krylov pass and updates the state.
//   FIN_INIT : beta = ||r0||, scale[0] = 1/beta, cols = 0, done if beta == 0
//   FIN_MV   : dots_i = scale_i * sum conj(V_i) w
//   FIN_ORTH1: H(i, jj) = dots_i (first round), dots_i = second-round products
//   FIN_ORTH2: H(i, jj) += dots_i, H(jj+1, jj) = ||w||, next scale; on breakdown
//              (||w|| <= tol beta) or at jj + 1 == m the Hessenberg least squares.
template <int KV>
__global__ __launch_bounds__(FBLOCK) void k_krylov_finalize(const double* __restrict__ partials, int nblk, int op,
                                                            int jj, int m, KrylovScal* K, double tol) {
    __shared__ double red[(FBLOCK / 64) * KV];
    __shared__ double sums[KV];
    if (op != FIN_INIT && K->done) return;
    const int kcount = (op == FIN_MV || op == FIN_ORTH1) ? 2 * (jj + 1) : 1;
    final_sum<KV>(partials, nblk, kcount, red, sums);
    if (threadIdx.x != 0) return;
    if (op == FIN_INIT) {
        double b = sqrt(sums[0]);
        K->beta = b;
        K->m = m;
        K->cols = 0;
        K->done = (b == 0.0 || !isfinite(b)) ? 1 : 0;
        K->scale[0] = b > 0.0 ? 1.0 / b : 0.0;
        if (K->done)
            for (int q = 0; q < MAXM; ++q) K->y[2 * q] = K->y[2 * q + 1] = 0.0;
    } else if (op == FIN_MV) {
        for (int i = 0; i <= jj; ++i) {
            double s = K->scale[i];
            K->dots[2 * i] = s * sums[2 * i];
            K->dots[2 * i + 1] = s * sums[2 * i + 1];
        }
    } else if (op == FIN_ORTH1) {
        for (int i = 0; i <= jj; ++i) {
            Hp(K, i, jj)[0] = K->dots[2 * i];
            Hp(K, i, jj)[1] = K->dots[2 * i + 1];
            double s = K->scale[i];
            K->dots[2 * i] = s * sums[2 * i];
            K->dots[2 * i + 1] = s * sums[2 * i + 1];
        }
    } else {
        for (int i = 0; i <= jj; ++i) {
            Hp(K, i, jj)[0] += K->dots[2 * i];
            Hp(K, i, jj)[1] += K->dots[2 * i + 1];
        }
        double hn = sqrt(sums[0]);
        Hp(K, jj + 1, jj)[0] = hn;
        Hp(K, jj + 1, jj)[1] = 0.0;
        K->cols = jj + 1;
        if (!isfinite(hn)) {
            K->done = 2;
            for (int q = 0; q < MAXM; ++q) K->y[2 * q] = K->y[2 * q + 1] = 0.0;
        } else if (hn <= tol * K->beta || jj + 1 == K->m) {
            ks_least_squares(K, jj + 1);
            K->done = 1;
        } else {
            K->scale[jj + 1] = 1.0 / hn;
        }
    }
}

// x = x0 + sum_{i < cols} y_i scale_i V_i  (x0 == nullptr: 0; x may alias x0).
template <typename T, int NV>
__global__ __launch_bounds__(BLOCK) void k_krylov_combine(size_t N, VecSet<T> V, const KrylovScal* K,
                                                          const cplx<T>* x0, cplx<T>* x) {
    const int cols = K->cols;
    cplx<T> c[NV];
#pragma unroll
    for (int i = 0; i < NV; ++i) {
        if (i < cols) {
            double s = K->scale[i];
            c[i] = mk<T>(T(K->y[2 * i] * s), T(K->y[2 * i + 1] * s));
        } else {
            c[i] = cplx<T>{};
        }
    }
    for (size_t p = blockIdx.x * (size_t)BLOCK + threadIdx.x; p < N; p += (size_t)gridDim.x * BLOCK) {
        cplx<T> v = x0 ? x0[p] : cplx<T>{};
#pragma unroll
        for (int i = 0; i < NV; ++i)
            if (i < cols) v = v + c[i] * V.v[i][p];
        x[p] = v;
    }
}

}  // namespace helm
