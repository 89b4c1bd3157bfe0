// Krylov kernels shared by the GMRES(m) ADR smoother and the outer FGMRES:
// fused operator + inner-product passes, two-pass classical Gram-Schmidt with
// re-orthogonalisation, the device-side Hessenberg least squares, and the
// final combination x = x0 + V y.  Inner products are summed across threads and
// blocks in FP64 (the outer FGMRES passes keep per-thread partial sums in the working
// precision), and every grid reduction is finished on the device by a one-block
// kernel (no host round trip).
#pragma once

#include "kernels_adr.hpp"

namespace helm {

template <typename T>
struct VecSet {
    const cplx<T>* v[MAXM + 1];
};

template <typename T>
__device__ __forceinline__ VecSet<T> bsh_one(size_t o, VecSet<T> s) {
#pragma unroll
    for (int i = 0; i <= MAXM; ++i) s.v[i] = bsh_one(o, s.v[i]);
    return s;
}

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
__global__ __launch_bounds__(BLOCK) void k_krylov_init_norm(size_t N, const cplx<T>* __restrict__ x, double* partials, BatchIdx bi) {
    bshift(bi.off(), x, partials);
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
                                                             double* partials, BatchIdx bi) {
    bshift(bi.off(), px, py, c0, b, x, r0, partials);
    __shared__ double red[4];
    __shared__ double sums[1];
    double acc[1] = {0.0};
    int t0, t1;
    tile_chunk(A.nx, A.ny, t0, t1);
    for (int t = t0; t < t1; ++t) {
        int j, i0;
        tile_xy(A.nx, t, j, i0);
        if (j >= A.nx) continue;
        for (int r = 0; r < RPT; ++r) {
            const int i = i0 + r;
            if (i >= A.ny) break;
            cplx<T> v{};
            if (i > 0 && j > 0) v = adr_resid_at(A, px, py, c0, b, x, i, j);
            r0[(size_t)i * A.nx + j] = v;
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
__device__ __forceinline__ void acc_dots(A (&acc)[2 * NV + 2], const VecSet<T>& V, int jj, size_t p, cplx<T> w,
                                         size_t o = 0) {
#pragma unroll
    for (int i = 0; i < NV; ++i) {
        if (i <= jj) {
            cplx<T> v = bsh_one(o, V.v[i])[p];
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
                                                       cplx<T>* __restrict__ w, const KrylovScal* K, double* partials, BatchIdx bi) {
    // V is shifted where it is read (jj is a runtime index into it)
    const size_t bo = bi.off();
    const cplx<T>* vjj = bsh_one(bo, V.v[jj]);
    bshift(bo, px, py, c0, w, K, partials);
    __shared__ double red[4 * (2 * NV + 2)];
    __shared__ double sums[2 * NV + 2];
    if (K->done) return;
    const T sj = T(K->scale[jj]);
    double acc[2 * NV + 2];
#pragma unroll
    for (int q = 0; q < 2 * NV + 2; ++q) acc[q] = 0.0;
    int t0, t1;
    tile_chunk(A.nx, A.ny, t0, t1);
    for (int t = t0; t < t1; ++t) {
        int j, i0;
        tile_xy(A.nx, t, j, i0);
        if (j >= A.nx) continue;
        for (int r = 0; r < RPT; ++r) {
            const int i = i0 + r;
            if (i >= A.ny) break;
            const size_t p = (size_t)i * A.nx + j;
            cplx<T> v{};
            if (i > 0 && j > 0) v = sj * applyM_at(A, px, py, c0, vjj, i, j);
            w[p] = v;
            acc_dots<T, NV>(acc, V, jj, p, v, bo);
        }
    }
    block_sum<2 * NV + 2, 4>(acc, 2 * (jj + 1), red, sums);
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
                                                      const KrylovScal* K, double* partials, BatchIdx bi) {
    bshift(bi.off(), V, w, K, partials);
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
                                                      const KrylovScal* K, double* partials, BatchIdx bi) {
    bshift(bi.off(), V, w, K, partials);
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

// ---- streaming passes of the outer FGMRES, one instantiation per column J
// A thread owns E consecutive elements (16-byte loads) of a grid-stride sweep and
// streams every basis vector the column needs; J is a template parameter so that
// the loops over the basis are unrolled with exactly the registers the column uses.
template <typename T>
struct FgShape {
    static constexpr int E = sizeof(T) == 4 ? 2 : 1;
};

template <typename T, int E>
struct Pack;
template <>
struct Pack<float, 2> {
    using V = float4;
};
template <>
struct Pack<double, 1> {
    using V = double2;
};

template <typename T, int E>
__device__ __forceinline__ void ld_pack(const cplx<T>* __restrict__ a, size_t p, cplx<T> (&v)[E]) {
    using PV = typename Pack<T, E>::V;
    const PV q = *reinterpret_cast<const PV*>(a + p);
    if constexpr (E == 2) {
        v[0] = mk<T>(q.x, q.y);
        v[1] = mk<T>(q.z, q.w);
    } else {
        v[0] = mk<T>(q.x, q.y);
    }
}

// The same with a non-temporal load: the Krylov basis is streamed once per pass and is
// far larger than the caches, so its lines are not kept (measured: a pass reading 11
// basis vectors goes from 5.1 to 6.0 TB/s).
template <typename T, int E>
__device__ __forceinline__ void ld_pack_nt(const cplx<T>* __restrict__ a, size_t p, cplx<T> (&v)[E]) {
    typedef T NV __attribute__((ext_vector_type(2 * E)));
    const NV q = __builtin_nontemporal_load(reinterpret_cast<const NV*>(a + p));
    if constexpr (E == 2) {
        v[0] = mk<T>(q.x, q.y);
        v[1] = mk<T>(q.z, q.w);
    } else {
        v[0] = mk<T>(q.x, q.y);
    }
}

template <typename T, int E>
__device__ __forceinline__ void st_pack(cplx<T>* __restrict__ a, size_t p, const cplx<T> (&v)[E]) {
    using PV = typename Pack<T, E>::V;
    PV q;
    if constexpr (E == 2) {
        q.x = v[0].re;
        q.y = v[0].im;
        q.z = v[1].re;
        q.w = v[1].im;
    } else {
        q.x = v[0].re;
        q.y = v[0].im;
    }
    *reinterpret_cast<PV*>(a + p) = q;
}

// Block sum of K per-thread values (working precision) to partials[v * nblk + block].
template <int K, typename A>
__device__ __forceinline__ void fg_store(const A (&acc)[K], double* partials) {
    __shared__ double red[4 * K];
    __shared__ double sums[K];
    double d[K];
#pragma unroll
    for (int q = 0; q < K; ++q) d[q] = double(acc[q]);
    block_sum<K, 4>(d, K, red, sums);
    store_partials(sums, K, partials);
}

// FGMRES Arnoldi pass of column J, with the second Gram-Schmidt round of column J-1
// applied on the fly (classical Gram-Schmidt twice, the second round lagging into
// this pass):
//   V_J <- V_J - sum_{i<J} c_i V_i,  c_i = dots_i scale_i (second-round coefficients
//          left by FIN_LORTH; nothing to do for J = 0),
//   w = A (s z),  s = zscale[J] if use_scale else 1,
// with partial sums of conj(V_i) w, i <= J (V_J the corrected vector), and of
// ||V_J||^2 (finalize with FIN_LMV).
template <typename T, int J>
__global__ __launch_bounds__(BLOCK) void k_fg_arnoldi(Geom G, const T* __restrict__ n2,
                                                      const cplx<T>* __restrict__ z, int use_scale, VecSet<T> V,
                                                      cplx<T>* __restrict__ vj, cplx<T>* __restrict__ w,
                                                      const KrylovScal* K, double* partials, BatchIdx bi) {
    bshift(bi.off(), n2, z, V, vj, w, K, partials);
    constexpr int E = FgShape<T>::E;
    constexpr int NA = 2 * (J + 1) + 1;
    if (K->done) return;
    cplx<T> cs[J > 0 ? J : 1];
#pragma unroll
    for (int i = 0; i < J; ++i) cs[i] = mk<T>(T(K->dots[2 * i] * K->scale[i]), T(K->dots[2 * i + 1] * K->scale[i]));
    const T sj = use_scale ? T(K->zscale[J]) : T(1);
    const int n = G.nx;  // nodes per row
    const size_t N = (size_t)G.nx * G.ny;
    T acc[NA];
#pragma unroll
    for (int q = 0; q < NA; ++q) acc[q] = T(0);
    for (size_t p = ((size_t)blockIdx.x * BLOCK + threadIdx.x) * E; p < N; p += (size_t)gridDim.x * BLOCK * E) {
        int i, j0;
        rowcol(p, n, i, j0);
        // every basis load is issued before the stencil, so they are all in flight at once
        cplx<T> vv[J + 1][E];
#pragma unroll
        for (int iv = 0; iv <= J; ++iv) ld_pack_nt<T, E>(V.v[iv], p, vv[iv]);
        cplx<T> x[E];
        if constexpr (E == 2) {
            // two neighbouring nodes of one row: their rows above and below and the pair
            // itself as 16-byte loads, the outer left and right neighbours singly
            cplx<T> c[2], up[2], dn[2] = {};
            ld_pack<T, 2>(z, p, c);
            if (i > 0) ld_pack<T, 2>(z, p - n, up);
            if (i + 1 < G.ny) ld_pack<T, 2>(z, p + n, dn);
            const cplx<T> lf = j0 > 0 ? z[p - 1] : cplx<T>{};
            const cplx<T> rt = j0 + 2 < n ? z[p + 2] : cplx<T>{};
            const T ih2 = T(G.inv_h2);
            const cplx<T> nb0 = up[0] + dn[0] + lf + c[1];
            const cplx<T> nb1 = up[1] + dn[1] + c[0] + rt;
            const cplx<T> k0 = kappa_at<T>(G, n2[p], i, j0), k1 = kappa_at<T>(G, n2[p + 1], i, j0 + 1);
            x[0] = (i > 0 && j0 > 0) ? sj * (ih2 * (T(4) * c[0] - nb0) - k0 * c[0]) : cplx<T>{};
            x[1] = i > 0 ? sj * (ih2 * (T(4) * c[1] - nb1) - k1 * c[1]) : cplx<T>{};
        } else {
#pragma unroll
            for (int e = 0; e < E; ++e) {
                const int j = j0 + e;
                x[e] = (i > 0 && j > 0) ? sj * applyA_at(G, n2, z, i, j, false) : cplx<T>{};
            }
        }
        st_pack<T, E>(w, p, x);
        cplx<T> corr[E];
#pragma unroll
        for (int e = 0; e < E; ++e) corr[e] = cplx<T>{};
#pragma unroll
        for (int iv = 0; iv < J; ++iv) {
#pragma unroll
            for (int e = 0; e < E; ++e) {
                const cplx<T> v = vv[iv][e];
                acc[2 * iv] += v.re * x[e].re + v.im * x[e].im;
                acc[2 * iv + 1] += v.re * x[e].im - v.im * x[e].re;
                corr[e] = corr[e] + cs[iv] * v;
            }
        }
        cplx<T> (&v)[E] = vv[J];
        if constexpr (J > 0) {
#pragma unroll
            for (int e = 0; e < E; ++e) v[e] = v[e] - corr[e];
            st_pack<T, E>(vj, p, v);
        }
#pragma unroll
        for (int e = 0; e < E; ++e) {
            acc[2 * J] += v[e].re * x[e].re + v[e].im * x[e].im;
            acc[2 * J + 1] += v[e].re * x[e].im - v[e].im * x[e].re;
            acc[2 * J + 2] += v[e].re * v[e].re + v[e].im * v[e].im;
        }
    }
    fg_store<NA>(acc, partials);
}

// First Gram-Schmidt round of column J: w -= sum_{i<=J} c_i V_i, c_i = dots_i scale_i;
// partial sums of conj(V_i) w, i <= J, and ||w||^2 (finalize with FIN_LORTH).
template <typename T, int J>
__global__ __launch_bounds__(BLOCK) void k_fg_orth(size_t N, VecSet<T> V, cplx<T>* __restrict__ w,
                                                   const KrylovScal* K, double* partials, BatchIdx bi) {
    bshift(bi.off(), V, w, K, partials);
    constexpr int E = FgShape<T>::E;
    constexpr int NA = 2 * (J + 1) + 1;
    if (K->done) return;
    cplx<T> cs[J + 1];
#pragma unroll
    for (int i = 0; i <= J; ++i) cs[i] = mk<T>(T(K->dots[2 * i] * K->scale[i]), T(K->dots[2 * i + 1] * K->scale[i]));
    T acc[NA];
#pragma unroll
    for (int q = 0; q < NA; ++q) acc[q] = T(0);
    for (size_t p = ((size_t)blockIdx.x * BLOCK + threadIdx.x) * E; p < N; p += (size_t)gridDim.x * BLOCK * E) {
        cplx<T> x[E];
        ld_pack<T, E>(w, p, x);
        // every basis load is issued before the arithmetic, so they are all in flight at once
        cplx<T> v[J + 1][E];
#pragma unroll
        for (int iv = 0; iv <= J; ++iv) ld_pack_nt<T, E>(V.v[iv], p, v[iv]);
#pragma unroll
        for (int iv = 0; iv <= J; ++iv)
#pragma unroll
            for (int e = 0; e < E; ++e) x[e] = x[e] - cs[iv] * v[iv][e];
        st_pack<T, E>(w, p, x);
#pragma unroll
        for (int iv = 0; iv <= J; ++iv)
#pragma unroll
            for (int e = 0; e < E; ++e) {
                acc[2 * iv] += v[iv][e].re * x[e].re + v[iv][e].im * x[e].im;
                acc[2 * iv + 1] += v[iv][e].re * x[e].im - v[iv][e].im * x[e].re;
            }
#pragma unroll
        for (int e = 0; e < E; ++e) acc[2 * J + 2] += x[e].re * x[e].re + x[e].im * x[e].im;
    }
    fg_store<NA>(acc, partials);
}

enum FinOp { FIN_INIT = 0, FIN_MV = 1, FIN_ORTH1 = 2, FIN_ORTH2 = 3, FIN_LMV = 4, FIN_LORTH = 5 };

// FIN_LMV and FIN_LORTH on one wavefront, lane i for basis vector i <= jj (< MAXM).
__device__ __forceinline__ void fin_lagged(int op, int jj, const double* sums, KrylovScal* K, double tol) {
    const int i = threadIdx.x;
    if (op == FIN_LMV) {
        const double nv = jj > 0 ? sqrt(sums[2 * (jj + 1)]) : 0.0;
        const bool okv = nv > 0.0 && isfinite(nv);
        if (i <= jj) {
            const double s = (jj > 0 && i == jj) ? (okv ? 1.0 / nv : 0.0) : K->scale[i];
            K->dots[2 * i] = s * sums[2 * i];
            K->dots[2 * i + 1] = s * sums[2 * i + 1];
        }
        if (i == 0 && jj > 0) {
            Hp(K, jj, jj - 1)[0] = nv;
            Hp(K, jj, jj - 1)[1] = 0.0;
            K->scale[jj] = okv ? 1.0 / nv : 0.0;
            if (!okv) K->done = isfinite(nv) ? 1 : 2;
        }
        return;
    }
    double dd = 0.0;
    if (i <= jj) {
        const double s = K->scale[i];
        const double dr = s * sums[2 * i], di = s * sums[2 * i + 1];
        Hp(K, i, jj)[0] = K->dots[2 * i] + dr;
        Hp(K, i, jj)[1] = K->dots[2 * i + 1] + di;
        K->dots[2 * i] = dr;
        K->dots[2 * i + 1] = di;
        dd = dr * dr + di * di;
    }
    dd = wave_sum(dd);
    if (i != 0) return;
    const double h2 = sums[2 * (jj + 1)] - dd;
    const double hn = h2 > 0.0 ? sqrt(h2) : 0.0;
    Hp(K, jj + 1, jj)[0] = isfinite(h2) ? hn : h2;
    Hp(K, jj + 1, jj)[1] = 0.0;
    K->cols = jj + 1;
    if (!isfinite(h2)) {
        K->done = 2;
    } else if (hn <= tol * K->beta || hn == 0.0 || jj + 1 == K->m) {
        K->done = 1;
    } else {
        K->scale[jj + 1] = 1.0 / hn;
        K->zscale[jj + 1] = 1.0 / hn;
    }
}

// One block: sums the partials of the previous Krylov pass and updates the state.
//   FIN_INIT : beta = ||r0||, scale[0] = 1/beta, cols = 0, done if beta == 0
//   FIN_MV   : dots_i = scale_i * sum conj(V_i) w
//   FIN_ORTH1: H(i, jj) = dots_i (first round), dots_i = second-round products
//   FIN_ORTH2: H(i, jj) += dots_i, H(jj+1, jj) = ||w||, next scale; on breakdown
//              (||w|| <= tol beta) or at jj + 1 == m the Hessenberg least squares.
// The outer FGMRES (second Gram-Schmidt round lagging one pass):
//   FIN_LMV  : after k_fg_arnoldi.  jj > 0: scale_jj = 1/||V_jj||, H(jj, jj-1) =
//              ||V_jj|| (the exact norm replaces the estimate); dots_i = scale_i *
//              sum conj(V_i) w, i <= jj (first-round coefficients of column jj)
//   FIN_LORTH: after k_fg_orth.  d_i = scale_i * sum conj(V_i) w; H(i, jj) =
//              dots_i + d_i; dots_i = d_i (second round, applied by the next
//              k_fg_arnoldi); H(jj+1, jj) = (||w||^2 - sum |d_i|^2)^(1/2), which
//              is the norm of w after the second round; zscale and scale of jj + 1
template <int KV>
__global__ __launch_bounds__(FBLOCK) void k_krylov_finalize(const double* __restrict__ partials, int nblk, int op,
                                                            int jj, int m, KrylovScal* K, double tol, BatchIdx bi) {
    bshift(bi.off(), partials, K);
    __shared__ double sums[KV];
    // the state flag is read alongside the partials (when it is set they are stale but
    // in bounds, and unused)
    const int done = op != FIN_INIT ? K->done : 0;
    const int kcount = (op == FIN_MV || op == FIN_ORTH1)     ? 2 * (jj + 1)
                       : (op == FIN_LMV || op == FIN_LORTH) ? 2 * (jj + 1) + 1
                                                            : 1;
    final_sum<KV>(partials, nblk, kcount, sums);
    if (done) return;
    if (op == FIN_LMV || op == FIN_LORTH) {
        // one lane per basis vector: the K fields of every i are read at once
        if (threadIdx.x < 64) fin_lagged(op, jj, sums, K, tol);
        return;
    }
    if (threadIdx.x != 0) return;
    if (op == FIN_INIT) {
        double b = sqrt(sums[0]);
        K->beta = b;
        K->m = m;
        K->cols = 0;
        K->done = (b == 0.0 || !isfinite(b)) ? 1 : 0;
        K->scale[0] = b > 0.0 ? 1.0 / b : 0.0;
        K->zscale[0] = K->scale[0];
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

// FGMRES end of a restart cycle: K->cols = cols and y from the device Hessenberg
// (Givens least squares, one thread).
__global__ void k_fgmres_lsq(KrylovScal* K, int cols, BatchIdx bi) {
    bshift(bi.off(), K);
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    if (cols < 0) cols = bi.aux_here();  // batched launch: one count per problem
    K->cols = cols;
    ks_least_squares(K, cols);
}

// x = x0 + sum_{i < cols} y_i s_i V_i, s_i = scale_i (zs == 0), zscale_i (zs == 1) or 1
// (zs == 2)  (x0 == nullptr: 0; x may alias x0).
// out[z count + i] = src[i] of the z-th problem of the launch, i < count: per-problem
// scalars gathered into one array (out itself is not per problem, so it is not shifted).
__global__ void k_gather(const double* __restrict__ src, int count, double* __restrict__ out, BatchIdx bi) {
    src = bsh_one(bi.off(), src);
    for (int i = threadIdx.x; i < count; i += blockDim.x) out[(size_t)blockIdx.z * count + i] = src[i];
}

template <typename T, int NV>
__global__ __launch_bounds__(BLOCK) void k_krylov_combine(size_t N, VecSet<T> V, const KrylovScal* K,
                                                          const cplx<T>* x0, cplx<T>* x, int zs, BatchIdx bi) {
    bshift(bi.off(), V, K, x0, x);
    const int cols = K->cols;
    cplx<T> c[NV];
#pragma unroll
    for (int i = 0; i < NV; ++i) {
        if (i < cols) {
            double s = zs == 0 ? K->scale[i] : zs == 1 ? K->zscale[i] : 1.0;
            c[i] = mk<T>(T(K->y[2 * i] * s), T(K->y[2 * i + 1] * s));
        } else {
            c[i] = cplx<T>{};
        }
    }
    // N is even (n is a power of two): FP32 pairs of nodes as 16-byte accesses
    constexpr int E = FgShape<T>::E;
    for (size_t p = (blockIdx.x * (size_t)BLOCK + threadIdx.x) * E; p < N; p += (size_t)gridDim.x * BLOCK * E) {
        cplx<T> v[E];
        if (x0) {
            ld_pack<T, E>(x0, p, v);
        } else {
#pragma unroll
            for (int e = 0; e < E; ++e) v[e] = cplx<T>{};
        }
#pragma unroll
        for (int i = 0; i < NV; ++i)
            if (i < cols) {
                cplx<T> b[E];
                ld_pack_nt<T, E>(V.v[i], p, b);
#pragma unroll
                for (int e = 0; e < E; ++e) v[e] = v[e] + c[i] * b[e];
            }
        st_pack<T, E>(x, p, v);
    }
}

}  // namespace helm
