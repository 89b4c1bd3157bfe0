// GMRES(m) smoother for the ADR operator in s-step form (m <= 4).
//
// GMRES(m) from x0 returns x = x0 + z, z in span{r0, M r0, ..., M^{m-1} r0}, that
// minimises ||r0 - M z||.  With K_j = M^j r0 this is the least-squares problem
// min_c || K_0 - sum_{j=1..m} c_j K_j ||, and then x = x0 + sum_j c_j K_{j-1}.
// The Krylov vectors are never stored; each pass rebuilds them:
//   pass 1 (k_sstep_gram):    K_0..K_m, Gram matrix G = K^H K (FP64 partial sums)
//   k_sstep_solve:            the partials summed (one wavefront per Gram entry), then
//                             the normalised Cholesky solve of the normal
//                             equations for c (one block)
//   pass 2 (k_sstep_combine): K_0..K_{m-1} again, x_out = x0 + sum c_j K_{j-1}
// The normalised monomial basis of the ADR operator is well conditioned for
// m <= 4 (condition numbers of 5-40 measured on the workloads), so the normal
// equations lose at most about three digits of FP64 accuracy.
//
// Both passes march: one wavefront owns a strip of 64 consecutive columns and
// walks down the rows of one segment, one row per step (S steps for S - 2H rows).  Lane l holds column
// j = jb - H + l, where [jb, jb + 64 - 2H) are the strip's own columns and H is
// the number of operator applications between the loaded fields and the last
// Krylov vector (the halo).  At the step that loads row q, K_j is produced on row
// q - j - D (D = 1 when K_0 = b - M x0 needs one application itself), so every
// operand row is already in registers: up/down neighbours come from register
// windows of the last rows of every field, left/right neighbours from the
// adjacent lanes (DPP lane shifts).  There is no LDS and no barrier; only the 2H
// halo columns and the 2H warm-up rows of a segment are computed twice.
#pragma once

#include <type_traits>

#include "kernels_krylov.hpp"

namespace helm {

// The value held by lane l - 1 (lane_prev) or lane l + 1 (lane_next) of the
// wavefront; 0 where that lane does not exist.
__device__ __forceinline__ float lane_prev(float v) {
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0x138 /* wave_shr:1 */, 0xF, 0xF, true));
}
__device__ __forceinline__ float lane_next(float v) {
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0x130 /* wave_shl:1 */, 0xF, 0xF, true));
}
__device__ __forceinline__ double lane_prev(double v) {
    const unsigned long long u = (unsigned long long)__double_as_longlong(v);
    const unsigned lo = (unsigned)__builtin_amdgcn_mov_dpp((int)(unsigned)u, 0x138, 0xF, 0xF, true);
    const unsigned hi = (unsigned)__builtin_amdgcn_mov_dpp((int)(unsigned)(u >> 32), 0x138, 0xF, 0xF, true);
    return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}
__device__ __forceinline__ double lane_next(double v) {
    const unsigned long long u = (unsigned long long)__double_as_longlong(v);
    const unsigned lo = (unsigned)__builtin_amdgcn_mov_dpp((int)(unsigned)u, 0x130, 0xF, 0xF, true);
    const unsigned hi = (unsigned)__builtin_amdgcn_mov_dpp((int)(unsigned)(u >> 32), 0x130, 0xF, 0xF, true);
    return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}
template <typename T>
__device__ __forceinline__ cplx<T> lane_prev(cplx<T> v) {
    return {lane_prev(v.re), lane_prev(v.im)};
}
template <typename T>
__device__ __forceinline__ cplx<T> lane_next(cplx<T> v) {
    return {lane_next(v.re), lane_next(v.im)};
}

// f(std::integral_constant<int, i>) for i = 0..N-1, unrolled at compile time.
template <int N, int I = 0, typename F>
__device__ __forceinline__ void static_for(F&& f) {
    if constexpr (I < N) {
        f(std::integral_constant<int, I>{});
        static_for<N, I + 1>(f);
    }
}

// a[p] addressed as a uniform base plus a 32-bit byte offset (every level array is
// below 4 GiB), which the hardware adds itself (no 64-bit address arithmetic).
template <typename V>
__device__ __forceinline__ V ld_off(const V* __restrict__ a, unsigned p) {
    return *reinterpret_cast<const V*>(reinterpret_cast<const char*>(a) + p * (unsigned)sizeof(V));
}
template <typename V>
__device__ __forceinline__ void st_off(V* __restrict__ a, unsigned p, V v) {
    *reinterpret_cast<V*>(reinterpret_cast<char*>(a) + p * (unsigned)sizeof(V)) = v;
}

// Upwind ADR stencil of one node with its constant factors folded in:
//   M a = C a_c - l sum_nb a_nb - i sum_nb g_nb a_nb,
//   l = 1/h^2,  C = c0 + 4 l - i g_c,  g = 2 sigma k / (2h) * (upwind weight of the node).
// Off the unknowns every factor is zero (l included), so M a = 0 there.
template <typename T>
struct UpCoef {
    T gw, ge, gs, gn;  // west (j-1), east (j+1), south (i-1), north (i+1)
    T cr, ci;          // C
    T nl;              // -1/h^2
};

// fx, fy, c0 must be zero off the unknowns (ok == false).
template <typename T>
__device__ __forceinline__ UpCoef<T> up_coef(const AdrGeom& A, T fx, T fy, cplx<T> c0, bool ok) {
    const T a = T(A.inv_2h) * T(A.two_sk);
    const T ax = fabs(fx), ay = fabs(fy);
    UpCoef<T> k;
    const T l = ok ? T(A.inv_h2) : T(0);
    k.nl = -l;
    k.gw = -a * (fx + ax);
    k.ge = a * (fx - ax);
    k.gs = -a * (fy + ay);
    k.gn = a * (fy - ay);
    k.cr = c0.re + T(4) * l;
    k.ci = c0.im - a * (T(2) * (ax + ay));
    return k;
}

// One accumulation chain per component, every neighbour value entering through its own
// multiply-add (signs as operand modifiers).
template <typename T>
__device__ __forceinline__ cplx<T> up_apply(const UpCoef<T>& k, cplx<T> c, cplx<T> w, cplx<T> e, cplx<T> s,
                                            cplx<T> n) {
    T re = k.cr * c.re;
    T im = k.cr * c.im;
    re = fma(-k.ci, c.im, re);
    im = fma(k.ci, c.re, im);
    re = fma(k.nl, s.re, re);
    im = fma(k.nl, s.im, im);
    re = fma(k.nl, n.re, re);
    im = fma(k.nl, n.im, im);
    re = fma(k.nl, w.re, re);
    im = fma(k.nl, w.im, im);
    re = fma(k.nl, e.re, re);
    im = fma(k.nl, e.im, im);
    re = fma(k.gs, s.im, re);
    im = fma(-k.gs, s.re, im);
    re = fma(k.gn, n.im, re);
    im = fma(-k.gn, n.re, im);
    re = fma(k.gw, w.im, re);
    im = fma(-k.gw, w.re, im);
    re = fma(k.ge, e.im, re);
    im = fma(-k.ge, e.re, im);
    return {re, im};
}

// Strip/segment geometry of the marching passes.  GRAM: the pass builds K_0..K_M
// (else K_0..K_{M-1}).
template <int M, bool X0, bool GRAM, int XH = 0, int EP = -1, int WR = 8>
struct March {
    static constexpr int D = X0 ? 1 : 0;
    static constexpr int NK = GRAM ? M : M - 1;  // last Krylov vector built
    static constexpr int H = NK + D + XH;        // halo of the loaded fields (XH: rows and
                                                 // columns beyond its own that a unit emits)
    static constexpr int TXW = 64 - 2 * H;       // columns owned by one strip
    static constexpr int W = WR;                 // rows kept per field (ring of registers, <= 8)
    // Steps after its own step that a loaded row is still read: x0 by K_0 of the next
    // row (and by the combination NK + D rows later), b by K_0, and the fields an
    // epilogue loads with the row by the emit of that row (EP = 0) or of the next one
    // (EP = 1; EP < 0: no such fields).  Rows are loaded as far ahead as the ring of W
    // registers allows.
    static constexpr int LAST0 = X0 ? (GRAM ? 2 : (NK + D > 2 ? NK + D : 2)) : 1;
    static constexpr int LAST = EP >= 0 && NK + D + EP > LAST0 ? NK + D + EP : LAST0;
    static constexpr int P = W - 1 - LAST;       // rows loaded ahead of the row they feed
    static_assert(P >= 1, "register ring too short for the halo");
    // A unit marches S steps (S a multiple of W) over a segment of S - 2H rows.
    __host__ __device__ static int rows(int S) { return S - 2 * H; }
    __host__ __device__ static int strips(int nx) { return (nx - 2) / TXW + 1; }
    __host__ __device__ static int units(int nx, int ny, int S) { return strips(nx) * ((ny - 2) / rows(S) + 1); }
};

// No fields beyond those of the Krylov vectors.
struct NoExtra {
    __device__ void init(int, bool, int, int) {}
    template <int SL>
    __device__ void load(int) {}
};

// Shared body of both passes.  Segments march down (DIR = +1) or up (DIR = -1) in
// turn, so that the warm-up rows two vertically adjacent units share are read by both at
// about the same time (at their starts or at their ends) and the second read hits L2.
// Per step: prefetch row q + DIR P (and ex's fields of it), fold the stencil of row q,
// then K_0 (X0: on row q - DIR) and K_1..K_NK on the rows behind it; the finished row
// r = q - DIR (NK + D) is handed to emit(r, slot, k, dir) (k[j] = K_j on row r; slot: the
// std::integral_constant ring position of row r; dir: std::integral_constant DIR) for
// the unit's rows and XH rows beyond them on either side.
template <typename T, int M, bool X0, bool GRAM, int XH, int EP, int DIR, int WR, typename Extra, typename Emit>
__device__ __forceinline__ void sstep_march_dir(const AdrGeom& A, int S, const T* __restrict__ px,
                                                const T* __restrict__ py, const cplx<T>* __restrict__ c0,
                                                const cplx<T>* __restrict__ b, const cplx<T>* __restrict__ x0,
                                                int j, bool colok, int rb, int re, cplx<T> (&xr)[8], Extra& ex,
                                                Emit& emit) {
    using Mc = March<M, X0, GRAM, XH, EP, WR>;
    constexpr int H = Mc::H, D = Mc::D, NK = Mc::NK, W = Mc::W, P = Mc::P;
    const int nx = A.nx, ny = A.ny;
    // first row loaded: the segment's rows plus H warm-up rows on the side it starts from
    const int q0 = DIR > 0 ? rb - H : rb + Mc::rows(S) - 1 + H;

    cplx<T> bw[W], kw[NK + 1][W];  // kw[NK] only holds the current row
    T fxw[W], fyw[W];
    cplx<T> cw0[W];
    UpCoef<T> cw[W];
#pragma unroll
    for (int s = 0; s < W; ++s) {
        xr[s] = cplx<T>{};
        bw[s] = cplx<T>{};
        fxw[s] = fyw[s] = T(0);
        cw0[s] = cplx<T>{};
        cw[s] = UpCoef<T>{};
#pragma unroll
        for (int q = 0; q <= NK; ++q) kw[q][s] = cplx<T>{};
    }
    // Every load is issued unconditionally: off the unknowns the row or column is replaced
    // by 0, whose stored values are the zero ring of every field read here (px, py, c0, b
    // and x0 all hold 0 on row 0 and column 0).  A load under a lane condition would sit
    // in a branch, after which the compiler can only wait for every outstanding load,
    // which would stall the prefetch at every row.
    const int jcl = colok ? j : 0;
    auto load_row = [&](int r, cplx<T>& xv, cplx<T>& bv, T& fx, T& fy, cplx<T>& cv) {
        const int rcl = (r >= 1 && r <= ny - 1) ? r : 0;
        const unsigned p = (unsigned)(rcl * nx + jcl);
        if (X0) xv = ld_off(x0, p);
        bv = ld_off(b, p);
        fx = ld_off(px, p);
        fy = ld_off(py, p);
        cv = ld_off(c0, p);
    };
    // the neighbours of a ring row: the one loaded before it lies on the side the march
    // comes from (south when marching down), the one loaded after it on the other side
    auto apply = [&](const UpCoef<T>& k, cplx<T> c, cplx<T> before, cplx<T> after) {
        if constexpr (DIR > 0)
            return up_apply<T>(k, c, lane_prev(c), lane_next(c), before, after);
        else
            return up_apply<T>(k, c, lane_prev(c), lane_next(c), after, before);
    };
    static_for<P>([&](auto pc) {
        constexpr int s = decltype(pc)::value;
        load_row(q0 + DIR * s, xr[s], bw[s], fxw[s], fyw[s], cw0[s]);
        ex.template load<s>(q0 + DIR * s);
    });
    for (int t0 = 0; t0 < S; t0 += W) {
        static_for<W>([&](auto sc) {
            constexpr int s = decltype(sc)::value;
            const int q = q0 + DIR * (t0 + s);
            // prefetch row q + DIR P
            constexpr int s1 = (s + P) % W;
            load_row(q + DIR * P, xr[s1], bw[s1], fxw[s1], fyw[s1], cw0[s1]);
            ex.template load<s1>(q + DIR * P);
            cw[s] = up_coef<T>(A, fxw[s], fyw[s], cw0[s], q >= 1 && q <= ny - 1 && colok);
            // K_0 (zero off the unknowns: b and the stencil factors are)
            if constexpr (X0) {
                constexpr int sr = (s + W - 1) % W;
                kw[0][sr] = bw[sr] - apply(cw[sr], xr[sr], xr[(s + W - 2) % W], xr[s]);
            } else {
                kw[0][s] = bw[s];
            }
            // K_1..K_NK
            static_for<NK>([&](auto jc) {
                constexpr int jj = decltype(jc)::value + 1;
                constexpr int sr = (s + 2 * W - jj - D) % W;
                kw[jj][sr] = apply(cw[sr], kw[jj - 1][sr], kw[jj - 1][(sr + W - 1) % W], kw[jj - 1][(sr + 1) % W]);
            });
            const int r = q - DIR * (NK + D);
            if (r >= rb - XH && r <= re + XH) {
                constexpr int sr = (s + 2 * W - NK - D) % W;
                cplx<T> k[NK + 1];
#pragma unroll
                for (int jj = 0; jj <= NK; ++jj) k[jj] = kw[jj][sr];
                emit(r, std::integral_constant<int, sr>{}, k, std::integral_constant<int, DIR>{});
            }
        });
    }
}

// The unit of this wavefront (column j of lane, rows [rb, re]) and its march, down on even
// segments and up on odd ones.
template <typename T, int M, bool X0, bool GRAM, int XH, int EP, int WR = 8, typename Extra, typename Emit>
__device__ __forceinline__ void sstep_march(const AdrGeom& A, int S, const T* __restrict__ px,
                                            const T* __restrict__ py, const cplx<T>* __restrict__ c0,
                                            const cplx<T>* __restrict__ b, const cplx<T>* __restrict__ x0,
                                            int& jcol, int& rb, int& re, cplx<T> (&xr)[8], Extra& ex,
                                            Emit&& emit) {
    using Mc = March<M, X0, GRAM, XH, EP>;
    constexpr int H = Mc::H;
    const int nx = A.nx, ny = A.ny;
    const int lane = threadIdx.x;
    const int ns = Mc::strips(nx);
    const int u = xcd_remap(blockIdx.x, gridDim.x);  // neighbouring units on one XCD
    const int sg = u / ns, st = u - sg * ns;
    const int j = 1 + st * Mc::TXW - H + lane;
    jcol = j;
    const bool colok = j >= 1 && j <= nx - 1;
    const int R = Mc::rows(S);
    rb = 1 + sg * R;
    re = rb + R - 1 < ny - 1 ? rb + R - 1 : ny - 1;
    ex.init(j, colok, nx, ny);
    if (sg & 1)
        sstep_march_dir<T, M, X0, GRAM, XH, EP, -1, WR>(A, S, px, py, c0, b, x0, j, colok, rb, re, xr, ex, emit);
    else
        sstep_march_dir<T, M, X0, GRAM, XH, EP, 1, WR>(A, S, px, py, c0, b, x0, j, colok, rb, re, xr, ex, emit);
}

// acc += the Gram entries of one node's K_0..K_M (layout of k_sstep_gram), in FP64.
template <typename T, int M>
__device__ __forceinline__ void gram_add(double (&acc)[(M + 1) * (M + 1)], const cplx<T> (&k)[M + 1]) {
    double kr[M + 1], ki[M + 1];
#pragma unroll
    for (int i = 0; i <= M; ++i) {
        kr[i] = double(k[i].re);
        ki[i] = double(k[i].im);
    }
    int o = M + 1;
#pragma unroll
    for (int i = 0; i <= M; ++i) {
        acc[i] = fma(ki[i], ki[i], fma(kr[i], kr[i], acc[i]));
#pragma unroll
        for (int jv = i + 1; jv <= M; ++jv) {
            acc[o] = fma(ki[i], ki[jv], fma(kr[i], kr[jv], acc[o]));
            acc[o + 1] = fma(-ki[i], kr[jv], fma(kr[i], ki[jv], acc[o + 1]));
            o += 2;
        }
    }
}

// Pass 1: per-wavefront Gram sums of K_0..K_M over the unit's own nodes, to
// partials[v * gridDim.x + blockIdx.x].  Layout of the NG doubles: G(i,i) real for
// i = 0..M, then G(i,j), i < j, as (re, im).  One wavefront per block.
template <typename T, int M, bool X0>
__global__ __launch_bounds__(64) void k_sstep_gram(AdrGeom A, int S, const T* __restrict__ px,
                                                   const T* __restrict__ py, const cplx<T>* __restrict__ c0,
                                                   const cplx<T>* __restrict__ b, const cplx<T>* __restrict__ x0,
                                                   double* __restrict__ partials, BatchIdx bi) {
    bshift(bi.off(), px, py, c0, b, x0, partials);
    using Mc = March<M, X0, true>;
    constexpr int NG = (M + 1) * (M + 1);
    // FP64 products: the unscaled powers M^j K_0 span many decades (|M| ~ 8/h^2)
    double acc[NG];
#pragma unroll
    for (int q = 0; q < NG; ++q) acc[q] = 0.0;
    const int lane = threadIdx.x;
    int j, rb, re;
    cplx<T> xr[8];
    const bool own_lane = lane >= Mc::H && lane < 64 - Mc::H;
    NoExtra ex;
    sstep_march<T, M, X0, true, 0, -1>(A, S, px, py, c0, b, x0, j, rb, re, xr, ex,
                                       [&](int r, auto, const cplx<T>(&k)[M + 1], auto) {
        (void)r;
        if (!(own_lane && j <= A.nx - 1)) return;
        gram_add<T, M>(acc, k);
    });
#pragma unroll
    for (int v = 0; v < NG; ++v) {
        const double sum = wave_sum(acc[v]);
        if (lane == 0) partials[(size_t)v * gridDim.x + blockIdx.x] = sum;
    }
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
        // reciprocals up front: one thread runs this, so the serial chain of divisions
        // and square roots is what it costs
        double d[M + 1], rd[M + 1];
#pragma unroll
        for (int i = 0; i <= M; ++i) {
            d[i] = sqrt(gr[i][i]);
            rd[i] = d[i] > 0 ? 1.0 / d[i] : 0.0;
        }
        // normalised normal equations N c' = r, N(i,j) = G(i,j)/(d_i d_j), r(i) = G(i,0)/(d_i d_0)
        double Lr[M][M], Li[M][M], il[M];
#pragma unroll
        for (int i = 0; i < M; ++i)
#pragma unroll
            for (int j = 0; j < M; ++j) {
                const double sc = rd[i + 1] * rd[j + 1];
                Lr[i][j] = gr[i + 1][j + 1] * sc;
                Li[i][j] = gi[i + 1][j + 1] * sc;
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
            il[j] = 1.0 / lj;
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
                Lr[i][j] = sr * il[j];
                Li[i][j] = si * il[j];
            }
        }
        double zr[M], zi[M];
#pragma unroll
        for (int i = 0; i < M; ++i) {  // L z = r  (rows >= cols give zero)
            const double sc = rd[i + 1] * rd[0];
            double sr = gr[i + 1][0] * sc, si = gi[i + 1][0] * sc;
#pragma unroll
            for (int q = 0; q < i; ++q) {
                sr -= Lr[i][q] * zr[q] - Li[i][q] * zi[q];
                si -= Lr[i][q] * zi[q] + Li[i][q] * zr[q];
            }
            zr[i] = i < cols ? sr * il[i] : 0.0;
            zi[i] = i < cols ? si * il[i] : 0.0;
        }
#pragma unroll
        for (int i = M - 1; i >= 0; --i) {  // L^H c' = z
            double sr = zr[i], si = zi[i];
#pragma unroll
            for (int q = i + 1; q < M; ++q) {
                sr -= Lr[q][i] * zr[q] + Li[q][i] * zi[q];
                si -= Lr[q][i] * zi[q] - Li[q][i] * zr[q];
            }
            zr[i] = i < cols ? sr * il[i] : 0.0;
            zi[i] = i < cols ? si * il[i] : 0.0;
        }
#pragma unroll
        for (int i = 0; i < M; ++i) {  // c_j = c'_j d_0 / d_j
            const double sc = i < cols ? d[0] * rd[i + 1] : 0.0;
            yr[i] = zr[i] * sc;
            yi[i] = zi[i] * sc;
        }
    }
}

// Reduction of the Gram partials and the coefficient solve in one block of SOLVE_THREADS
// threads: wavefront v sums partials[v * nblk + b] over b (fixed order; the loads of a
// lane are issued in batches of up to SOLVE_BATCH before the adds), then thread 0 solves the
// normal equations and writes K->y (c_j of K_{j-1}, zero for dropped columns), K->cols,
// K->beta = ||K_0|| and K->done (1; 2 if the norm is not finite).
constexpr int SOLVE_THREADS = 1024, SOLVE_BATCH = 32;

// Lane's share of a row of nblk partials: row[lane], row[lane + 64], ... added in order,
// the loads issued SB at a time before the adds.
template <int SB>
__device__ __forceinline__ double lane_row_sum(const double* __restrict__ row, int nblk, int lane) {
    double acc = 0.0;
    for (int b0 = 0; b0 < nblk; b0 += 64 * SB) {
        double t[SB];
#pragma unroll
        for (int k = 0; k < SB; ++k) {
            const int bb = b0 + k * 64 + lane;
            t[k] = bb < nblk ? row[bb] : 0.0;
        }
#pragma unroll
        for (int k = 0; k < SB; ++k) acc += t[k];
    }
    return acc;
}

template <int M>
__global__ __launch_bounds__(SOLVE_THREADS) void k_sstep_solve(const double* __restrict__ partials, int nblk,
                                                               double breakdown_tol, KrylovScal* K, BatchIdx bi) {
    bshift(bi.off(), partials, K);
    constexpr int NG = (M + 1) * (M + 1), NW = SOLVE_THREADS / 64;
    __shared__ double sums[NG];
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
    for (int v = wv; v < NG; v += NW) {
        const double* __restrict__ row = partials + (size_t)v * nblk;
        // a batch no longer than the row (the same sums: the loads left out read zeros)
        double acc = nblk <= 64     ? lane_row_sum<1>(row, nblk, lane)
                     : nblk <= 256  ? lane_row_sum<4>(row, nblk, lane)
                     : nblk <= 1024 ? lane_row_sum<16>(row, nblk, lane)
                                    : lane_row_sum<SOLVE_BATCH>(row, nblk, lane);
        acc = wave_sum(acc);
        if (lane == 0) sums[v] = acc;
    }
    __syncthreads();
    if (threadIdx.x != 0) return;
    double g[NG];
#pragma unroll
    for (int q = 0; q < NG; ++q) g[q] = sums[q];
    double yr[M], yi[M], beta;
    int cols;
    sstep_small_solve<M>(g, breakdown_tol, yr, yi, cols, beta);
    K->beta = beta;
#pragma unroll
    for (int j = 0; j < M; ++j) {
        K->y[2 * j] = yr[j];
        K->y[2 * j + 1] = yi[j];
    }
    K->cols = cols;
    K->done = isfinite(beta) ? 1 : 2;
}

// What pass 2 does with x = x0 + sum c_j K_{j-1} (X0 only for the last two): write
// it (EPI_X); add it, re-modulated, to the level-2 iterate (EPI_MOD: u_out = u + x
// e^{i theta}); or do that and also demodulate the next ADR right-hand side from the
// updated iterate (EPI_MODRD: b_out = (g - A u_out) e^{-i theta}), which needs x one
// node beyond the unit, so that variant runs with one more halo row and column.
enum { EPI_X = 0, EPI_MOD = 1, EPI_MODRD = 2 };

// Level-2 fields of the modulated epilogues.
template <typename T>
struct ModArgs {
    Geom G;                   // wave geometry of level 2 (sizes as on the ADR level)
    const cplx<T>* car;       // carrier e^{i sigma k phi}
    const T* n2;              // n^2 on level 2 (EPI_MODRD)
    const cplx<T>* g;         // level-2 right-hand side (EPI_MODRD)
    const cplx<T>* u;         // level-2 iterate, read
    cplx<T>* uout;            // level-2 iterate, written (may be u for EPI_MOD)
    cplx<T>* bout;            // next ADR right-hand side (EPI_MODRD)
};

template <typename T>
__device__ __forceinline__ ModArgs<T> bsh_one(size_t o, ModArgs<T> a) {
    a.car = bsh_one(o, a.car);
    a.n2 = bsh_one(o, a.n2);
    a.g = bsh_one(o, a.g);
    a.u = bsh_one(o, a.u);
    a.uout = bsh_one(o, a.uout);
    a.bout = bsh_one(o, a.bout);
    return a;
}

// Rows of the level-2 fields, prefetched with the Krylov rows.
template <typename T, int EPI>
struct ModExtra {
    const ModArgs<T>& a;
    int j = 0, nx = 0, ny = 0;
    bool colok = false;
    cplx<T> cr[8];
    cplx<T> uu[8];
    cplx<T> gg[EPI == EPI_MODRD ? 8 : 1];
    T nn[EPI == EPI_MODRD ? 8 : 1];
    __device__ explicit ModExtra(const ModArgs<T>& args) : a(args) {}
    __device__ void init(int jj, bool ok, int nlx, int nly) {
        j = jj;
        colok = ok;
        nx = nlx;
        ny = nly;
    }
    template <int SL>
    __device__ void load(int r) {
        if constexpr (EPI != EPI_X) {
            // unconditional, as the Krylov rows: off the unknowns row / column 0, where u is 0
            // (the update there is u + 0 * car) and g, n2 feed no stored residual
            const int rcl = (r >= 1 && r <= ny - 1) ? r : 0;
            const unsigned p = (unsigned)(rcl * nx + (colok ? j : 0));
            cr[SL] = ld_off(a.car, p);
            uu[SL] = ld_off(a.u, p);
            if constexpr (EPI == EPI_MODRD) {
                gg[SL] = ld_off(a.g, p);
                nn[SL] = ld_off(a.n2, p);
            }
        }
    }
};

// Pass 2: x = x0 + sum_{j=1..cols} c_j K_{j-1} on the unit's own nodes with the
// coefficients of k_sstep_solve, then the epilogue EPI; also writes the zero ring
// (row 0, column 0) of every array it writes in full.
template <typename T, int M, bool X0, int EPI>
__global__ __launch_bounds__(64) void k_sstep_combine(AdrGeom A, int S, const T* __restrict__ px,
                                                      const T* __restrict__ py, const cplx<T>* __restrict__ c0,
                                                      const cplx<T>* __restrict__ b, const cplx<T>* __restrict__ x0,
                                                      const KrylovScal* __restrict__ K, cplx<T>* __restrict__ xout,
                                                      ModArgs<T> mod, BatchIdx bi) {
    bshift(bi.off(), px, py, c0, b, x0, K, xout, mod);
    static_assert(EPI == EPI_X || X0, "the modulated epilogues follow the post-smoother");
    constexpr int XH = EPI == EPI_MODRD ? 1 : 0;
    constexpr int EP = EPI == EPI_X ? -1 : EPI == EPI_MOD ? 0 : 1;
    // FP64 with the modulated epilogue: a ring of six rows (one row of prefetch), so that
    // the registers allow two wavefronts per SIMD
    constexpr int WR = (sizeof(T) == 8 && EPI == EPI_MODRD) ? 6 : 8;
    using Mc = March<M, X0, false, XH, EP, WR>;
    constexpr int W = Mc::W;
    const int lane = threadIdx.x;
    const int nx = A.nx, ny = A.ny;
    cplx<T> c[M];
#pragma unroll
    for (int q = 0; q < M; ++q) c[q] = mk<T>(T(K->y[2 * q]), T(K->y[2 * q + 1]));
    int j, rb, re;
    cplx<T> xr[8];
    const bool own_lane = lane >= Mc::H && lane < 64 - Mc::H;
    if constexpr (EPI != EPI_MOD) {
        // the ring: column 0 of the segment's rows (strip 0), row 0 (segment 0)
        const int ns = Mc::strips(nx);
        int u = blockIdx.x;
        const int nb = gridDim.x;
        u = xcd_remap(u, nb);
        const int sg = u / ns, st = u - sg * ns;
        const int jj = 1 + st * Mc::TXW - Mc::H + lane;
        const int R = Mc::rows(S);
        const int r0 = 1 + sg * R, r1 = r0 + R - 1 < ny - 1 ? r0 + R - 1 : ny - 1;
        auto zero_at = [&](size_t p) {
            if constexpr (EPI == EPI_X) {
                xout[p] = cplx<T>{};
            } else {
                mod.uout[p] = cplx<T>{};
                mod.bout[p] = cplx<T>{};
            }
        };
        if (jj == 0)
            for (int r = r0; r <= r1; ++r) zero_at((size_t)r * nx);
        if (sg == 0 && ((own_lane && jj <= nx - 1) || jj == 0)) zero_at((size_t)jj);
    }
    auto xval = [&](auto slot, const cplx<T>(&k)[M]) {
        constexpr int sr = decltype(slot)::value;
        cplx<T> v = X0 ? xr[sr] : cplx<T>{};
#pragma unroll
        for (int q = 0; q < M; ++q) v = v + c[q] * k[q];
        return v;
    };
    if constexpr (EPI == EPI_X) {
        NoExtra ex;
        sstep_march<T, M, X0, false, 0, EP>(A, S, px, py, c0, b, x0, j, rb, re, xr, ex,
                                            [&](int r, auto slot, const cplx<T>(&k)[M], auto) {
                                            const cplx<T> v = xval(slot, k);
                                            if (own_lane && j <= nx - 1) st_off(xout, (unsigned)(r * nx + j), v);
                                        });
    } else if constexpr (EPI == EPI_MOD) {
        ModExtra<T, EPI> ex(mod);
        sstep_march<T, M, X0, false, 0, EP>(A, S, px, py, c0, b, x0, j, rb, re, xr, ex,
                                            [&](int r, auto slot, const cplx<T>(&k)[M], auto) {
                                            constexpr int sr = decltype(slot)::value;
                                            const cplx<T> v = xval(slot, k);
                                            if (own_lane && j <= nx - 1)
                                                st_off(mod.uout, (unsigned)(r * nx + j), ex.uu[sr] + v * ex.cr[sr]);
                                        });
    } else {
        ModExtra<T, EPI> ex(mod);
        cplx<T> un[W];  // updated iterate of the emitted rows
        const Geom& G = mod.G;
        const T ih2 = T(G.inv_h2);
        sstep_march<T, M, X0, false, 1, EP, WR>(
            A, S, px, py, c0, b, x0, j, rb, re, xr, ex, [&](int r, auto slot, const cplx<T>(&k)[M], auto dirc) {
                constexpr int sr = decltype(slot)::value;
                constexpr int s1 = (sr + W - 1) % W, s2 = (sr + W - 2) % W;
                const cplx<T> v = xval(slot, k);
                un[sr] = ex.uu[sr] + v * ex.cr[sr];
                const int ri = r - decltype(dirc)::value;  // the row emitted before this one
                if (ri >= rb && ri <= re) {
                    const cplx<T> cu = un[s1];
                    const cplx<T> w = lane_prev(cu), e = lane_next(cu);
                    const cplx<T> nb = ((un[s2] + un[sr]) + w) + e;
                    const cplx<T> lap = ih2 * (T(4) * cu - nb);
                    const cplx<T> kap = kappa_at<T>(G, ex.nn[s1], ri, j);
                    const cplx<T> res = ex.gg[s1] - (lap - kap * cu);
                    if (own_lane && j <= nx - 1) {
                        const unsigned p = (unsigned)(ri * nx + j);
                        st_off(mod.bout, p, res * conjg(ex.cr[s1]));
                        st_off(mod.uout, p, cu);
                    }
                }
            });
    }
}

// Pass 2 of a pre-smoother (x0 = 0) fused with the restriction of its residual:
// x = sum_j c_j K_{j-1} on the own nodes, and since b - M x = K_0 - sum_j c_j K_j the
// residual comes from one more Krylov vector instead of an application of M to x.  The
// unit emits one row and column beyond its own, weights each residual row across lanes
// (1 2 1) and, at every odd fine row whose neighbour emitted before it (2I) is its own, combines the last
// three rows (1 2 1) / 16 into the coarse row I of rc (nx/2 x ny/2 nodes) at the own
// even columns.  Also writes the zero rings of x and rc.
template <typename T, int M>
__global__ __launch_bounds__(64) void k_sstep_combine_rr(AdrGeom A, int S, const T* __restrict__ px,
                                                         const T* __restrict__ py, const cplx<T>* __restrict__ c0,
                                                         const cplx<T>* __restrict__ b,
                                                         const KrylovScal* __restrict__ K, cplx<T>* __restrict__ xout,
                                                         cplx<T>* __restrict__ rc, BatchIdx bi) {
    bshift(bi.off(), px, py, c0, b, K, xout, rc);
    using Mc = March<M, false, true, 1, -1>;
    constexpr int W = Mc::W;
    const int lane = threadIdx.x;
    const int nx = A.nx, ny = A.ny, ncx = nx / 2;
    cplx<T> c[M];
#pragma unroll
    for (int q = 0; q < M; ++q) c[q] = mk<T>(T(K->y[2 * q]), T(K->y[2 * q + 1]));
    const bool own_lane = lane >= Mc::H && lane < 64 - Mc::H;
    {
        const int ns = Mc::strips(nx);
        const int u = xcd_remap(blockIdx.x, gridDim.x);
        const int sg = u / ns, st = u - sg * ns;
        const int jj = 1 + st * Mc::TXW - Mc::H + lane;
        const int R = Mc::rows(S);
        const int r0 = 1 + sg * R, r1 = r0 + R - 1 < ny - 1 ? r0 + R - 1 : ny - 1;
        if (jj == 0) {
            for (int r = r0; r <= r1; ++r) xout[(size_t)r * nx] = cplx<T>{};
            for (int I = (r0 + 1) >> 1; 2 * I <= r1; ++I) rc[(size_t)I * ncx] = cplx<T>{};
        }
        if (sg == 0 && ((own_lane && jj <= nx - 1) || jj == 0)) {
            xout[jj] = cplx<T>{};
            if (!(jj & 1)) rc[jj >> 1] = cplx<T>{};
        }
    }
    int j, rb, re;
    cplx<T> xr[8];
    cplx<T> hr[W];  // residual rows weighted across lanes, by ring slot
    NoExtra ex;
    sstep_march<T, M, false, true, 1, -1>(A, S, px, py, c0, b, nullptr, j, rb, re, xr, ex,
                                          [&](int r, auto slot, const cplx<T>(&k)[M + 1], auto dirc) {
        constexpr int sr = decltype(slot)::value;
        constexpr int s1 = (sr + W - 1) % W, s2 = (sr + W - 2) % W;
        cplx<T> xv{};
        cplx<T> rv = k[0];
#pragma unroll
        for (int q = 0; q < M; ++q) {
            xv = xv + c[q] * k[q];
            rv = rv - c[q] * k[q + 1];
        }
        if (own_lane && j <= nx - 1 && r >= rb && r <= re) st_off(xout, (unsigned)(r * nx + j), xv);
        hr[sr] = (lane_prev(rv) + lane_next(rv)) + T(2) * rv;
        const int cm = r - decltype(dirc)::value;  // the middle one of the last three rows
        const int I = cm >> 1;
        if ((r & 1) && cm >= rb && cm <= re && I >= 1) {
            const cplx<T> v = T(1.0 / 16.0) * ((hr[s2] + hr[sr]) + T(2) * hr[s1]);
            if (own_lane && !(j & 1) && j <= nx - 1) st_off(rc, (unsigned)(I * ncx + (j >> 1)), v);
        }
    });
}

// ------------------------------------------------------------------ overlapped-tile form
// On the small ADR levels one marching unit per SIMD cannot hide its row-to-row
// latency.  There a block of BLOCK threads owns a TT x TT tile of unknowns and builds
// the Krylov vectors on the tile and a ring of H nodes around it, one vector per
// barrier, in LDS.  Values outside the ring are taken as zero, so the ring's values
// are wrong by one more node per operator application and the tile's own values are
// exact after the H applications; the region's border nodes are simply set to zero.
template <int M, bool X0, bool GRAM, int TT, int XH = 0>
struct Tile {
    static constexpr int D = X0 ? 1 : 0;
    static constexpr int NK = GRAM ? M : M - 1;
    static constexpr int H = NK + D + XH;  // XH: ring of exact values beyond the tile
    static constexpr int RW = TT + 2 * H;  // region width
    static constexpr int NR = RW * RW;
    static constexpr int NPT = (NR + BLOCK - 1) / BLOCK;  // region nodes per thread
    // tiles along a side of m nodes, and over a level of nx x ny nodes
    __host__ __device__ static int per_side(int m) { return (m - 2) / TT + 1; }
    __host__ __device__ static int tiles(int nx, int ny) { return per_side(nx) * per_side(ny); }
};

// Shared body of the tile passes; buf: 2 NR values of LDS.  emit(q, gi, gj, own, x0, k)
// for every node of the tile and its ring of XH nodes (q: region index; own: a node of
// the tile inside the grid; k[j] = K_j there, exact, and 0 off the grid; x0 the iterate
// there, 0 without X0).  The last step reads only buffer (NK - 1 + D) % 2, so emit may
// write the other one, (NK + D) % 2.
template <typename T, int M, bool X0, bool GRAM, int TT, int XH = 0, typename Emit>
__device__ __forceinline__ void sstep_tile(const AdrGeom& A, int ti, int tj, const T* __restrict__ px,
                                           const T* __restrict__ py, const cplx<T>* __restrict__ c0,
                                           const cplx<T>* __restrict__ b, const cplx<T>* __restrict__ x0,
                                           cplx<T>* buf, Emit&& emit) {
    using Tg = Tile<M, X0, GRAM, TT, XH>;
    constexpr int RW = Tg::RW, NR = Tg::NR, NPT = Tg::NPT, H = Tg::H, NK = Tg::NK;
    const int nx = A.nx, ny = A.ny;
    const int i0 = 1 + ti * TT - H, j0 = 1 + tj * TT - H;  // region node (0, 0)
    const int tid = threadIdx.x;
    cplx<T> xv[NPT], bv[NPT], cv[NPT];
    T fx[NPT], fy[NPT];
    bool ok[NPT];
#pragma unroll
    for (int k = 0; k < NPT; ++k) {
        const int q = tid + k * BLOCK;
        const int ri = q / RW, rj = q - ri * RW;
        const int gi = i0 + ri, gj = j0 + rj;
        xv[k] = bv[k] = cv[k] = cplx<T>{};
        fx[k] = fy[k] = T(0);
        ok[k] = q < NR && gi >= 1 && gi <= ny - 1 && gj >= 1 && gj <= nx - 1;
        if (ok[k]) {
            const unsigned p = (unsigned)(gi * nx + gj);
            if constexpr (X0) xv[k] = ld_off(x0, p);
            bv[k] = ld_off(b, p);
            fx[k] = ld_off(px, p);
            fy[k] = ld_off(py, p);
            cv[k] = ld_off(c0, p);
        }
    }
    UpCoef<T> cf[NPT];
    bool inner[NPT];
#pragma unroll
    for (int k = 0; k < NPT; ++k) {
        const int q = tid + k * BLOCK;
        const int ri = q / RW, rj = q - ri * RW;
        cf[k] = up_coef<T>(A, fx[k], fy[k], cv[k], ok[k]);
        inner[k] = q < NR && ri >= 1 && ri <= RW - 2 && rj >= 1 && rj <= RW - 2;
    }
    auto apply = [&](const cplx<T>* src, int k) -> cplx<T> {
        const int q = tid + k * BLOCK;
        return up_apply<T>(cf[k], src[q], src[q - 1], src[q + 1], src[q - RW], src[q + RW]);
    };
    // K_j lives in buffer (j + D) % 2; x0 (X0) in buffer 0
    cplx<T> kv[NK + 1][NPT];
    if constexpr (X0) {
#pragma unroll
        for (int k = 0; k < NPT; ++k)
            if (tid + k * BLOCK < NR) buf[tid + k * BLOCK] = xv[k];
        __syncthreads();
#pragma unroll
        for (int k = 0; k < NPT; ++k) kv[0][k] = inner[k] ? bv[k] - apply(buf, k) : cplx<T>{};
    } else {
#pragma unroll
        for (int k = 0; k < NPT; ++k) kv[0][k] = bv[k];
    }
    static_for<NK>([&](auto jc) {
        constexpr int jj = decltype(jc)::value + 1;
        cplx<T>* src = buf + ((jj - 1 + Tg::D) % 2) * NR;
#pragma unroll
        for (int k = 0; k < NPT; ++k)
            if (tid + k * BLOCK < NR) src[tid + k * BLOCK] = kv[jj - 1][k];
        __syncthreads();
#pragma unroll
        for (int k = 0; k < NPT; ++k) kv[jj][k] = inner[k] ? apply(src, k) : cplx<T>{};
    });
#pragma unroll
    for (int k = 0; k < NPT; ++k) {
        const int q = tid + k * BLOCK;
        const int ri = q / RW, rj = q - ri * RW;
        const int gi = i0 + ri, gj = j0 + rj;
        if (q < NR && ri >= H - XH && ri < H + TT + XH && rj >= H - XH && rj < H + TT + XH) {
            const bool own = ri >= H && ri < H + TT && rj >= H && rj < H + TT && gi <= ny - 1 && gj <= nx - 1;
            cplx<T> kk[NK + 1];
#pragma unroll
            for (int jj = 0; jj <= NK; ++jj) kk[jj] = kv[jj][k];
            emit(q, gi, gj, own, xv[k], kk);
        }
    }
}

// Tile row ti and column tj of this block; per_row tiles along a row of the level.
__device__ __forceinline__ void tile_index(int per_row, int& ti, int& tj) {
    const int t = xcd_remap(blockIdx.x, gridDim.x);
    ti = t / per_row;
    tj = t - ti * per_row;
}

// Pass 1 in tile form: per-block Gram sums to partials[v * gridDim.x + blockIdx.x]
// (layout of k_sstep_gram); Tile<M, X0, true, TT>::tiles(nx, ny) blocks.
template <typename T, int M, bool X0, int TT>
__global__ __launch_bounds__(BLOCK) void k_sstep_gram_tile(AdrGeom A, const T* __restrict__ px,
                                                           const T* __restrict__ py,
                                                           const cplx<T>* __restrict__ c0,
                                                           const cplx<T>* __restrict__ b,
                                                           const cplx<T>* __restrict__ x0,
                                                           double* __restrict__ partials, BatchIdx bi) {
    bshift(bi.off(), px, py, c0, b, x0, partials);
    using Tg = Tile<M, X0, true, TT>;
    constexpr int NG = (M + 1) * (M + 1);
    __shared__ cplx<T> buf[2 * Tg::NR];
    __shared__ double red[(BLOCK / 64) * NG];
    __shared__ double sums[NG];
    double acc[NG];
#pragma unroll
    for (int q = 0; q < NG; ++q) acc[q] = 0.0;
    int ti, tj;
    tile_index(Tg::per_side(A.nx), ti, tj);
    sstep_tile<T, M, X0, true, TT>(A, ti, tj, px, py, c0, b, x0, buf,
                                   [&](int, int, int, bool own, cplx<T>, const cplx<T>(&k)[M + 1]) {
                                       if (own) gram_add<T, M>(acc, k);
                                   });
    block_sum<NG, BLOCK / 64>(acc, NG, red, sums);
    store_partials(sums, NG, partials);
}

// Pass 2 in tile form with the EPI_X epilogue: xout = x0 + sum c_j K_{j-1} on the own
// nodes, and the zero ring (row 0, column 0); Tile<M, X0, false, TT>::tiles(nx, ny) blocks.
template <typename T, int M, bool X0, int TT>
__global__ __launch_bounds__(BLOCK) void k_sstep_combine_tile(AdrGeom A, const T* __restrict__ px,
                                                              const T* __restrict__ py,
                                                              const cplx<T>* __restrict__ c0,
                                                              const cplx<T>* __restrict__ b,
                                                              const cplx<T>* __restrict__ x0,
                                                              const KrylovScal* __restrict__ K,
                                                              cplx<T>* __restrict__ xout, BatchIdx bi) {
    bshift(bi.off(), px, py, c0, b, x0, K, xout);
    using Tg = Tile<M, X0, false, TT>;
    __shared__ cplx<T> buf[2 * Tg::NR];
    const int nx = A.nx, ny = A.ny;
    cplx<T> c[M];
#pragma unroll
    for (int q = 0; q < M; ++q) c[q] = mk<T>(T(K->y[2 * q]), T(K->y[2 * q + 1]));
    int ti, tj;
    tile_index(Tg::per_side(nx), ti, tj);
    const int tid = threadIdx.x;
    if (tid < TT) {
        const int jr = 1 + tj * TT + tid, ir = 1 + ti * TT + tid;
        if (ti == 0 && jr <= nx - 1) xout[jr] = cplx<T>{};
        if (tj == 0 && ir <= ny - 1) xout[(size_t)ir * nx] = cplx<T>{};
        if (ti == 0 && tj == 0 && tid == 0) xout[0] = cplx<T>{};
    }
    sstep_tile<T, M, X0, false, TT>(A, ti, tj, px, py, c0, b, x0, buf,
                                    [&](int, int gi, int gj, bool own, cplx<T> xo, const cplx<T>(&k)[M]) {
                                        if (!own) return;
                                        cplx<T> v = X0 ? xo : cplx<T>{};
#pragma unroll
                                        for (int q = 0; q < M; ++q) v = v + c[q] * k[q];
                                        st_off(xout, (unsigned)(gi * nx + gj), v);
                                    });
}

// Tile form of k_sstep_combine_rr: x = sum_j c_j K_{j-1} on the tile, the residual
// K_0 - sum_j c_j K_j on the tile and a ring of one node (into the free LDS buffer),
// then its full weighting at the coarse nodes whose centre is a node of the tile (one
// per thread for 32 x 32 tiles), and the zero rings of x and rc.
template <typename T, int M, int TT>
__global__ __launch_bounds__(BLOCK) void k_sstep_combine_tile_rr(AdrGeom A, const T* __restrict__ px,
                                                                 const T* __restrict__ py,
                                                                 const cplx<T>* __restrict__ c0,
                                                                 const cplx<T>* __restrict__ b,
                                                                 const KrylovScal* __restrict__ K,
                                                                 cplx<T>* __restrict__ xout, cplx<T>* __restrict__ rc, BatchIdx bi) {
    bshift(bi.off(), px, py, c0, b, K, xout, rc);
    using Tg = Tile<M, false, true, TT, 1>;
    constexpr int RW = Tg::RW, H = Tg::H, TC = TT / 2;
    static_assert(TT % 2 == 0 && TC * TC <= BLOCK, "one coarse node per thread");
    __shared__ cplx<T> buf[2 * Tg::NR];
    const int nx = A.nx, ny = A.ny, ncx = nx / 2, ncy = ny / 2;
    cplx<T> c[M];
#pragma unroll
    for (int q = 0; q < M; ++q) c[q] = mk<T>(T(K->y[2 * q]), T(K->y[2 * q + 1]));
    int ti, tj;
    tile_index(Tg::per_side(nx), ti, tj);
    const int tid = threadIdx.x;
    if (tid < TT) {
        const int jr = 1 + tj * TT + tid, ir = 1 + ti * TT + tid;
        if (ti == 0 && jr <= nx - 1) xout[jr] = cplx<T>{};
        if (tj == 0 && ir <= ny - 1) xout[(size_t)ir * nx] = cplx<T>{};
        if (ti == 0 && tj == 0 && tid == 0) xout[0] = cplx<T>{};
    }
    if (tid < TC) {
        const int Jr = 1 + tj * TC + tid, Ir = 1 + ti * TC + tid;
        if (ti == 0 && Jr <= ncx - 1) rc[Jr] = cplx<T>{};
        if (tj == 0 && Ir <= ncy - 1) rc[(size_t)Ir * ncx] = cplx<T>{};
        if (ti == 0 && tj == 0 && tid == 0) rc[0] = cplx<T>{};
    }
    cplx<T>* res = buf + ((Tg::NK + Tg::D) % 2) * Tg::NR;
    sstep_tile<T, M, false, true, TT, 1>(A, ti, tj, px, py, c0, b, nullptr, buf,
                                         [&](int q, int gi, int gj, bool own, cplx<T>, const cplx<T>(&k)[M + 1]) {
                                             cplx<T> xv{};
                                             cplx<T> rv = k[0];
#pragma unroll
                                             for (int qq = 0; qq < M; ++qq) {
                                                 xv = xv + c[qq] * k[qq];
                                                 rv = rv - c[qq] * k[qq + 1];
                                             }
                                             if (own) st_off(xout, (unsigned)(gi * nx + gj), xv);
                                             res[q] = rv;
                                         });
    __syncthreads();
    // coarse node (I, J) = (1 + ti TC + ci, 1 + tj TC + cj): fine centre (2I, 2J) at region
    // row 2I - (1 + ti TT - H) = 1 + 2 ci + H, column likewise
    if (tid < TC * TC) {
        const int ci = tid / TC, cj = tid - ci * TC;
        const int I = 1 + ti * TC + ci, J = 1 + tj * TC + cj;
        if (I <= ncy - 1 && J <= ncx - 1) {
            const int l = (1 + 2 * ci + H) * RW + 1 + 2 * cj + H;
            const cplx<T> cc = res[l];
            const cplx<T> ud = ((res[l - RW] + res[l + RW]) + res[l - 1]) + res[l + 1];
            const cplx<T> dg = ((res[l - RW - 1] + res[l - RW + 1]) + res[l + RW - 1]) + res[l + RW + 1];
            st_off(rc, (unsigned)(I * ncx + J), T(1.0 / 16.0) * ((T(4) * cc + T(2) * ud) + dg));
        }
    }
}

// Tile form of pass 2 with the prolongation epilogue: x = x0 + sum_j c_j K_{j-1} on the
// tile and a ring of one node (LDS), then xf += P x (bilinear) on the fine nodes of the
// tile: fine rows and columns 2I and 2I + 1 of its coarse nodes, and row / column 1 on
// the first tiles (xf has 2 nx x 2 ny nodes; its zero ring is left alone).  x itself is
// not stored: its only use is this prolongation.
template <typename T, int M, bool X0, int TT>
__global__ __launch_bounds__(BLOCK) void k_sstep_combine_tile_pa(AdrGeom A, const T* __restrict__ px,
                                                                 const T* __restrict__ py,
                                                                 const cplx<T>* __restrict__ c0,
                                                                 const cplx<T>* __restrict__ b,
                                                                 const cplx<T>* __restrict__ x0,
                                                                 const KrylovScal* __restrict__ K,
                                                                 cplx<T>* __restrict__ xf, BatchIdx bi) {
    bshift(bi.off(), px, py, c0, b, x0, K, xf);
    using Tg = Tile<M, X0, false, TT, 1>;
    constexpr int RW = Tg::RW, H = Tg::H;
    __shared__ cplx<T> buf[2 * Tg::NR];
    const int nx = A.nx, ny = A.ny, nfx = 2 * nx;
    cplx<T> c[M];
#pragma unroll
    for (int q = 0; q < M; ++q) c[q] = mk<T>(T(K->y[2 * q]), T(K->y[2 * q + 1]));
    int ti, tj;
    tile_index(Tg::per_side(nx), ti, tj);
    cplx<T>* xs = buf + ((Tg::NK + Tg::D) % 2) * Tg::NR;
    sstep_tile<T, M, X0, false, TT, 1>(A, ti, tj, px, py, c0, b, x0, buf,
                                       [&](int q, int, int, bool, cplx<T> xo, const cplx<T>(&k)[M]) {
                                           cplx<T> v = X0 ? xo : cplx<T>{};
#pragma unroll
                                           for (int qq = 0; qq < M; ++qq) v = v + c[qq] * k[qq];
                                           xs[q] = v;
                                       });
    __syncthreads();
    const int Ia = 1 + ti * TT, Ib = Ia + TT - 1 < ny - 1 ? Ia + TT - 1 : ny - 1;
    const int Ja = 1 + tj * TT, Jb = Ja + TT - 1 < nx - 1 ? Ja + TT - 1 : nx - 1;
    const int f0 = ti == 0 ? 1 : 2 * Ia, f1 = 2 * Ib + 1;
    const int i0 = Ia - H, j0 = Ja - H;  // coarse node of region (0, 0)
    // fine columns in pairs (2J, 2J + 1) over the tile's coarse columns J, one read-modify-
    // write of both nodes per pair (16 bytes in FP32); column 1 alone on the first tiles
    const int NP = Jb - Ja + 1, FR = f1 - f0 + 1;
    for (int q = threadIdx.x; q < FR * NP; q += BLOCK) {
        const int fr = q / NP;
        const int f = f0 + fr, J = Ja + (q - fr * NP);
        const int I = f >> 1;
        const int l = (I - i0) * RW + (J - j0);
        cplx<T> ve, vo;  // columns 2J and 2J + 1
        if (!(f & 1)) {
            ve = xs[l];
            vo = T(0.5) * (xs[l] + xs[l + 1]);
        } else {
            ve = T(0.5) * (xs[l] + xs[l + RW]);
            vo = T(0.25) * (((xs[l] + xs[l + RW]) + xs[l + 1]) + xs[l + RW + 1]);
        }
        const unsigned p = (unsigned)(f * nfx + 2 * J);
        if constexpr (sizeof(T) == 4) {
            float4* a = reinterpret_cast<float4*>(reinterpret_cast<char*>(xf) + p * (unsigned)sizeof(cplx<T>));
            float4 w4 = *a;
            w4.x += ve.re;
            w4.y += ve.im;
            w4.z += vo.re;
            w4.w += vo.im;
            *a = w4;
        } else {
            st_off(xf, p, ld_off((const cplx<T>*)xf, p) + ve);
            st_off(xf, p + 1, ld_off((const cplx<T>*)xf, p + 1) + vo);
        }
    }
    if (tj == 0) {  // fine column 1: between coarse columns 0 (zero) and 1
        for (int fr = threadIdx.x; fr < FR; fr += BLOCK) {
            const int f = f0 + fr, I = f >> 1;
            const int l = (I - i0) * RW + (0 - j0);
            const cplx<T> v = (f & 1) ? T(0.25) * (((xs[l] + xs[l + RW]) + xs[l + 1]) + xs[l + RW + 1])
                                      : T(0.5) * (xs[l] + xs[l + 1]);
            const unsigned p = (unsigned)(f * nfx + 1);
            st_off(xf, p, ld_off((const cplx<T>*)xf, p) + v);
        }
    }
}

}  // namespace helm
