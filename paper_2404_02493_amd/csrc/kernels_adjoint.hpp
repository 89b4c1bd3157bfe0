// Reverse-mode kernels of the unrolled Wave-ADR cycle: the back-propagation of
// the training loss of Section 3.3 (eq. loss) through K cycles of Algorithm 1.
//
// Convention: for a real loss L the cotangent of a complex array x is
// xbar = dL/dRe(x) + i dL/dIm(x) (torch's convention), so a complex-linear map
// y = B x pulls back as xbar = B^H ybar, and a real parameter p that enters y
// receives Re <ybar, dy/dp>, with <a, b> = sum conj(a) b.
//
// The operators involved and their adjoints:
//   A   = -Delta_h - diag(kappa)        A^H = -Delta_h - diag(conj kappa)
//   R   full weighting                  R^T = P / 4  (P bilinear, P = 4 R^T)
//   M   upwind ADR operator (eq. ADR, eq. upwind); M^H gathers the conjugated
//       coefficients of the neighbouring rows (the stencil is not symmetric).
// Every kernel keeps the ring i = 0 or j = 0 at zero, as the forward kernels do.
#pragma once

#include "kernels_sstep.hpp"

namespace helm {

constexpr int GMAX = 6;  // largest GMRES dimension the adjoint supports

// State of one GMRES(m) call of the ADR smoother, recorded in the monomial Krylov
// basis k_1 = r0, k_{j+1} = M k_j / tau (tau only scales the basis), so that
// x = x0 + sum_j c_j k_j with c the least-squares solution of the normal equations
// (W^H W) c = W^H r0, W = tau [k_2 .. k_{m+1}].  All FP64.
struct GRec {
    double gram[(GMAX + 1) * (GMAX + 2)];  // column c (1-based): <k_i, k_c>, i <= c, at 2*(c(c-1)/2 + i-1)
    double c[2 * GMAX];
    double Lf[2 * GMAX * GMAX];            // Cholesky factor of the normalised W^H W (lower, row-major)
    double dsc[GMAX];                      // normalisation 1/sqrt(diag(W^H W))
    double cbar[2 * GMAX];                 // <k_j, xbar>
    double z[2 * GMAX];                    // (W^H W)^{-1} cbar
    double coef[2 * (GMAX + 1) * (GMAX + 2)];  // row r (0-based, kbar_{r+1}) over (xbar, k_1..k_{m+1})
    double one[2];                         // the coefficient row (1, 0): xbar alone
    int m;                                 // requested dimension
    int rank;                              // columns used (< m when the Krylov space is invariant)
    int zero;                              // r0 == 0: x = x0
    int pad;
};
constexpr int GCOEF_STRIDE = 2 * (GMAX + 2);

__device__ __forceinline__ int gram_off(int i, int c) { return 2 * (c * (c - 1) / 2 + i - 1); }

template <typename T>
__device__ __forceinline__ cplx<T> ldc(const cplx<T>* __restrict__ a, int i, int j, int nx, int ny) {
    if (i <= 0 || j <= 0 || i >= ny || j >= nx) return cplx<T>{};
    return a[(size_t)i * nx + j];
}

// Per-block sums of K accumulators into partials[v * nblk + block] (256 threads).
template <int K>
__device__ __forceinline__ void reduce_store(const double (&acc)[K], int kcount, double* partials) {
    __shared__ double red[4 * K];
    __shared__ double sums[K];
    block_sum<K, 4>(acc, kcount, red, sums);
    store_partials(sums, kcount, partials);
}

// acc[2q] + i acc[2q+1] += <k_q, y> = conj(k_q) y at one node, q < md (FP64 products).
// The reverse of a taped GMRES call needs <k_j, xbar> for its output cotangent xbar; the
// pass that produces xbar forms their per-block partials on the way (grid-stride over
// fb(nodes) blocks, the layout k_ga_prep reads).
template <typename T>
__device__ __forceinline__ void dots_add(double (&acc)[2 * GMAX], const VecSet<T>& Kd, int md, size_t p,
                                         cplx<T> y) {
#pragma unroll
    for (int q = 0; q < GMAX; ++q) {
        if (q < md) {
            const cplx<T> k = Kd.v[q][p];
            acc[2 * q] += double(k.re) * double(y.re) + double(k.im) * double(y.im);
            acc[2 * q + 1] += double(k.re) * double(y.im) - double(k.im) * double(y.re);
        }
    }
}

// Weight cotangents of up to WSLOTS reverse passes, summed in one launch: slot q holds the
// nblk[q] per-block partials of one pass at wpart + q * stride (the pass's reduce_store);
// wavefront q sums slot q (group_row_sum, the order of the finalize kernels), then
// wacc[level[q]] += that sum for q = 0, 1, ... (the order the passes ran in).
constexpr int WSLOTS = FBLOCK / 64;
struct WSlots {
    int n;
    int nblk[WSLOTS];
    int level[WSLOTS];
};
__global__ __launch_bounds__(FBLOCK) void k_wsum(const double* __restrict__ wpart, int stride, WSlots t,
                                                 double* __restrict__ wacc) {
    __shared__ double sums[WSLOTS];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    if (wv < t.n) {
        const double sv = group_row_sum(wpart + (size_t)wv * stride, t.nblk[wv], lane);
        if (lane == 0) sums[wv] = sv;
    }
    __syncthreads();
    if (threadIdx.x == 0)
        for (int q = 0; q < t.n; ++q) wacc[t.level[q]] += 1.0 * sums[q];
}

// ------------------------------------------------------------------ wave levels

// Jacobi sweep y = u + w D^{-1} (g - A u), D = 4/h^2 - kappa (eq. sjac), reversed:
//   ubar_out = ybar - w A^H (D^{-H} ybar),   wbar += Re <ybar, D^{-1} (g - A u)>.
template <typename T>
__global__ __launch_bounds__(BLOCK) void k_jacobi_adj(Geom G, const T* __restrict__ n2, const cplx<T>* __restrict__ g,
                                                      const cplx<T>* __restrict__ u, const cplx<T>* __restrict__ yb,
                                                      cplx<T>* __restrict__ ub, T w, double* partials) {
    const int n = G.nx;  // nodes per row
    const size_t N = (size_t)n * G.ny;
    double acc[1] = {0.0};
    auto dinv_h = [&](int a, int b) -> cplx<T> {  // ybar(a,b) / conj(D(a,b)), zero off the unknowns
        if (a <= 0 || b <= 0 || a >= G.ny || b >= n) return cplx<T>{};
        const size_t q = (size_t)a * n + b;
        cplx<T> kap = kappa_at<T>(G, n2[q], a, b);
        cplx<T> dh = mk<T>(T(4) * T(G.inv_h2) - kap.re, kap.im);  // conj(D)
        return cdiv(yb[q], dh);
    };
    for (size_t p = blockIdx.x * (size_t)BLOCK + threadIdx.x; p < N; p += (size_t)gridDim.x * BLOCK) {
        int i, j;
        rowcol(p, n, i, j);
        cplx<T> out{};
        if (i > 0 && j > 0) {
            cplx<T> kap = kappa_at<T>(G, n2[p], i, j);
            cplx<T> d = mk<T>(T(4) * T(G.inv_h2) - kap.re, -kap.im);
            cplx<T> res = resid_at(G, n2, g, u, i, j);
            cplx<T> q = cdiv(res, d);
            cplx<T> y = yb[p];
            acc[0] += double(y.re) * double(q.re) + double(y.im) * double(q.im);
            cplx<T> qc = dinv_h(i, j);
            cplx<T> nb = ((dinv_h(i - 1, j) + dinv_h(i + 1, j)) + dinv_h(i, j - 1)) + dinv_h(i, j + 1);
            cplx<T> ahq = T(G.inv_h2) * (T(4) * qc - nb) - conjg(kap) * qc;
            out = y - w * ahq;
        }
        ub[p] = out;
    }
    reduce_store<1>(acc, 1, partials);
}

// xc = s * R x (full weighting from the fine level of nx x ny nodes).
template <typename Tf, typename Tc>
__global__ __launch_bounds__(BLOCK) void k_restrict_scale(int nx, int ny, const cplx<Tf>* __restrict__ x,
                                                          cplx<Tc>* __restrict__ xc, double s) {
    const int ncx = nx / 2;
    const size_t N = (size_t)ncx * (ny / 2);
    for (size_t p = blockIdx.x * (size_t)BLOCK + threadIdx.x; p < N; p += (size_t)gridDim.x * BLOCK) {
        int I, J;
        rowcol(p, ncx, I, J);
        cplx<Tc> out{};
        if (I > 0 && J > 0) {
            const int fi = 2 * I, fj = 2 * J;
            auto X = [&](int a, int b) { return ccast<double>(ldc(x, a, b, nx, ny)); };
            c128 c = X(fi, fj);
            c128 e = ((X(fi - 1, fj) + X(fi + 1, fj)) + X(fi, fj - 1)) + X(fi, fj + 1);
            c128 dg = ((X(fi - 1, fj - 1) + X(fi - 1, fj + 1)) + X(fi + 1, fj - 1)) + X(fi + 1, fj + 1);
            c128 v = (s / 16.0) * ((4.0 * c + 2.0 * e) + dg);
            out = ccast<Tc>(v);
        }
        xc[p] = out;
    }
}

// k_restrict_scale on one precision with the per-block partials of <k_q, xc>, q < md
// (Kd: k_1..k_md on the coarse level), the dots of the reverse call that reads xc next.
// fb(coarse nodes) blocks.
template <typename T>
__global__ __launch_bounds__(BLOCK) void k_restrict_scale_dots(int nx, int ny, const cplx<T>* __restrict__ x,
                                                               cplx<T>* __restrict__ xc, double s, VecSet<T> Kd,
                                                               int md, double* __restrict__ partials) {
    const int ncx = nx / 2;
    const size_t N = (size_t)ncx * (ny / 2);
    double acc[2 * GMAX];
#pragma unroll
    for (int v = 0; v < 2 * GMAX; ++v) acc[v] = 0.0;
    for (size_t p = blockIdx.x * (size_t)BLOCK + threadIdx.x; p < N; p += (size_t)gridDim.x * BLOCK) {
        int I, J;
        rowcol(p, ncx, I, J);
        cplx<T> out{};
        if (I > 0 && J > 0) {
            const int fi = 2 * I, fj = 2 * J;
            auto X = [&](int a, int b) { return ccast<double>(ldc(x, a, b, nx, ny)); };
            c128 c = X(fi, fj);
            c128 e = ((X(fi - 1, fj) + X(fi + 1, fj)) + X(fi, fj - 1)) + X(fi, fj + 1);
            c128 dg = ((X(fi - 1, fj - 1) + X(fi - 1, fj + 1)) + X(fi + 1, fj - 1)) + X(fi + 1, fj + 1);
            c128 v = (s / 16.0) * ((4.0 * c + 2.0 * e) + dg);
            out = ccast<T>(v);
            dots_add(acc, Kd, md, p, out);
        }
        xc[p] = out;
    }
    if (md > 0) reduce_store<2 * GMAX>(acc, 2 * md, partials);
}

// Reverse of rc = R (g - A u) given rcbar on the coarse level: with t = P rcbar / 4,
//   gbar += t  (if gbar),   ubar -= A^H t  (if ubar).  In place on gbar and ubar.
template <typename Tc, typename Tf>
__global__ __launch_bounds__(BLOCK) void k_prolong_adj(Geom G, const Tf* __restrict__ n2,
                                                       const cplx<Tc>* __restrict__ rcbar, cplx<Tf>* __restrict__ ubar,
                                                       cplx<Tf>* __restrict__ gbar) {
    const int n = G.nx, ny = G.ny;  // n: nodes per row
    const size_t N = (size_t)n * ny;
    auto tq = [&](int a, int b) -> cplx<Tf> {
        if (a <= 0 || b <= 0 || a >= ny || b >= n) return cplx<Tf>{};
        return Tf(0.25) * prolong_at<Tc, Tf>(rcbar, n / 2, ny / 2, a, b);
    };
    for (size_t p = blockIdx.x * (size_t)BLOCK + threadIdx.x; p < N; p += (size_t)gridDim.x * BLOCK) {
        int i, j;
        rowcol(p, n, i, j);
        if (i == 0 || j == 0) continue;
        const cplx<Tf> t = tq(i, j);
        if (gbar) gbar[p] = gbar[p] + t;
        if (ubar) {
            cplx<Tf> kap = kappa_at<Tf>(G, n2[p], i, j);
            cplx<Tf> nb = ((tq(i - 1, j) + tq(i + 1, j)) + tq(i, j - 1)) + tq(i, j + 1);
            cplx<Tf> aht = Tf(G.inv_h2) * (Tf(4) * t - nb) - conjg(kap) * t;
            ubar[p] = ubar[p] - aht;
        }
    }
}

// gbar += t (if gbar);  ubar -= A^H t (if ubar).  In place.
template <typename T>
__global__ __launch_bounds__(BLOCK) void k_adj_ahsub(Geom G, const T* __restrict__ n2, const cplx<T>* __restrict__ t,
                                                     cplx<T>* __restrict__ ubar, cplx<T>* __restrict__ gbar) {
    const int n = G.nx;  // nodes per row
    const size_t N = (size_t)n * G.ny;
    for (size_t p = blockIdx.x * (size_t)BLOCK + threadIdx.x; p < N; p += (size_t)gridDim.x * BLOCK) {
        int i, j;
        rowcol(p, n, i, j);
        if (i == 0 || j == 0) continue;
        if (gbar) gbar[p] = gbar[p] + t[p];
        if (ubar) ubar[p] = ubar[p] - applyA_at(G, n2, t, i, j, true);
    }
}

// Chebyshev reverse, start of the primal + alpha-tangent recurrences on v:
//   r = v, rt = 0, d = v / theta, dt = v * dt0, s = d, st = dt.
template <typename T>
__global__ __launch_bounds__(BLOCK) void k_chebadj_start(size_t N, const cplx<T>* __restrict__ v, cplx<T>* __restrict__ r,
                                                         cplx<T>* __restrict__ rt, cplx<T>* __restrict__ d,
                                                         cplx<T>* __restrict__ dt, cplx<T>* __restrict__ s,
                                                         cplx<T>* __restrict__ st, T inv_theta, T dt0) {
    for (size_t p = blockIdx.x * (size_t)BLOCK + threadIdx.x; p < N; p += (size_t)gridDim.x * BLOCK) {
        const cplx<T> x = v[p];
        const cplx<T> dd = inv_theta * x, ddt = dt0 * x;
        r[p] = x;
        rt[p] = cplx<T>{};
        d[p] = dd;
        dt[p] = ddt;
        s[p] = dd;
        st[p] = ddt;
    }
}

// One step of both recurrences of the Chebyshev adjoint in one pass on a 64 x 16 tile:
// t1 = A d_in and t2 = A dt_in on the tile and a ring of one node in
// LDS (from d_in, dt_in on a ring of two), then at the tile's nodes
//   r -= A^H t1; rt -= A^H t2; d_out = c1 d + c2 r; dt_out = c1t d + c1 dt + c2t r + c2 rt;
//   s += d_out; st += dt_out.
// d_out, dt_out must not alias d_in, dt_in (neighbouring tiles still read them); their
// ring is written 0.  The LDS of d_in, dt_in is reused for t1, t2.  tiles_of(nx, ny)
// blocks of 64 x 4 threads.
template <typename T>
__global__ __launch_bounds__(BLOCK) void k_chebadj_fused(Geom G, const T* __restrict__ n2,
                                                         const cplx<T>* __restrict__ d_in,
                                                         const cplx<T>* __restrict__ dt_in, cplx<T>* __restrict__ d_out,
                                                         cplx<T>* __restrict__ dt_out, cplx<T>* __restrict__ r,
                                                         cplx<T>* __restrict__ rt, cplx<T>* __restrict__ s,
                                                         cplx<T>* __restrict__ st, T c1, T c2, T c1t, T c2t) {
    constexpr int DW = TX + 4, DH = TY + 4, HW = TX + 2, HH = TY + 2;
    constexpr int NQ1 = (HH * HW + BLOCK - 1) / BLOCK;
    __shared__ cplx<T> sa[DH * DW];  // d_in (ring 2), then t1 (ring 1, width HW)
    __shared__ cplx<T> sb[DH * DW];  // dt_in (ring 2), then t2
    __shared__ T sn[HH * HW];
    const int nx = G.nx, ny = G.ny;
    const T ih2 = T(G.inv_h2);
    int j, i0;
    tile_origin(nx, j, i0);
    const int jt = j - (int)threadIdx.x, it = i0 - (int)threadIdx.y * RPT;  // tile origin
    const int tid = threadIdx.x + threadIdx.y * TX;
    cplx<T> fa[TileRing<2>::NQ], fb[TileRing<2>::NQ];
    T fn[TileRing<1>::NQ];
    tile_fetch<2>(d_in, nx, ny, it, jt, fa);
    tile_fetch<2>(dt_in, nx, ny, it, jt, fb);
    tile_fetch<1>(n2, nx, ny, it, jt, fn);
    cplx<T> rv0[RPT], rtv0[RPT], dv0[RPT], dtv0[RPT];
#pragma unroll
    for (int rr = 0; rr < RPT; ++rr) {
        const int i = i0 + rr;
        rv0[rr] = rtv0[rr] = dv0[rr] = dtv0[rr] = cplx<T>{};
        if (i >= 1 && i < ny && j >= 1 && j < nx) {
            const size_t p = (size_t)i * nx + j;
            rv0[rr] = r[p];
            rtv0[rr] = rt[p];
            dv0[rr] = d_in[p];
            dtv0[rr] = dt_in[p];
        }
    }
    tile_store<2>(fa, sa);
    tile_store<2>(fb, sb);
    tile_store<1>(fn, sn);
    __syncthreads();
    cplx<T> t1r[NQ1], t2r[NQ1];
#pragma unroll
    for (int k = 0; k < NQ1; ++k) {  // t = A d on the tile and a ring of one
        const int q = tid + k * BLOCK;
        t1r[k] = t2r[k] = cplx<T>{};
        if (q >= HH * HW) continue;
        const int ri = q / HW, rj = q - ri * HW;
        const int gi = it - 1 + ri, gj = jt - 1 + rj;
        if (gi >= 1 && gj >= 1 && gi < ny && gj < nx) {
            const int l = (ri + 1) * DW + rj + 1;
            const cplx<T> kap = kappa_at<T>(G, sn[q], gi, gj);
            const cplx<T> ca = sa[l], cb = sb[l];
            t1r[k] = ih2 * (T(4) * ca - (((sa[l - DW] + sa[l + DW]) + sa[l - 1]) + sa[l + 1])) - kap * ca;
            t2r[k] = ih2 * (T(4) * cb - (((sb[l - DW] + sb[l + DW]) + sb[l - 1]) + sb[l + 1])) - kap * cb;
        }
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < NQ1; ++k) {
        const int q = tid + k * BLOCK;
        if (q < HH * HW) {
            sa[q] = t1r[k];
            sb[q] = t2r[k];
        }
    }
    __syncthreads();
    if (j >= nx) return;
#pragma unroll
    for (int rr = 0; rr < RPT; ++rr) {
        const int i = i0 + rr;
        if (i >= ny) break;
        const size_t p = (size_t)i * nx + j;
        if (i == 0 || j == 0) {  // the ring of the alternate buffers
            d_out[p] = cplx<T>{};
            dt_out[p] = cplx<T>{};
            continue;
        }
        const int l = (i - it + 1) * HW + (j - jt + 1);
        cplx<T> kap = kappa_at<T>(G, sn[l], i, j);
        kap.im = -kap.im;
        const cplx<T> a1 = sa[l], a2 = sb[l];
        const cplx<T> h1 = ih2 * (T(4) * a1 - (((sa[l - HW] + sa[l + HW]) + sa[l - 1]) + sa[l + 1])) - kap * a1;
        const cplx<T> h2 = ih2 * (T(4) * a2 - (((sb[l - HW] + sb[l + HW]) + sb[l - 1]) + sb[l + 1])) - kap * a2;
        const cplx<T> rv = rv0[rr] - h1, rtv = rtv0[rr] - h2;
        const cplx<T> dn = c1 * dv0[rr] + c2 * rv;
        const cplx<T> dtn = ((c1t * dv0[rr] + c1 * dtv0[rr]) + c2t * rv) + c2 * rtv;
        r[p] = rv;
        rt[p] = rtv;
        d_out[p] = dn;
        dt_out[p] = dtn;
        s[p] = s[p] + dn;
        st[p] = st[p] + dtn;
    }
}

// partial Re <a, A^H b>
template <typename T>
__global__ __launch_bounds__(BLOCK) void k_dot_ah(Geom G, const T* __restrict__ n2, const cplx<T>* __restrict__ a,
                                                  const cplx<T>* __restrict__ b, double* partials) {
    const int n = G.nx;  // nodes per row
    const size_t N = (size_t)n * G.ny;
    double acc[1] = {0.0};
    for (size_t p = blockIdx.x * (size_t)BLOCK + threadIdx.x; p < N; p += (size_t)gridDim.x * BLOCK) {
        int i, j;
        rowcol(p, n, i, j);
        if (i == 0 || j == 0) continue;
        const cplx<T> v = applyA_at(G, n2, b, i, j, true);
        const cplx<T> x = a[p];
        acc[0] += double(x.re) * double(v.re) + double(x.im) * double(v.im);
    }
    reduce_store<1>(acc, 1, partials);
}

// ------------------------------------------------------------------ ADR correction (level 2)

// Reverse of u' = u + a e^{i theta} (car = e^{i theta}):  abar = e^{-i theta} ubar',
// thbar += Re <ubar', i a e^{i theta}> = -Im(conj(ubar') a e^{i theta}); with md > 0 also
// the per-block partials of <k_q, abar>, q < md (Kd: k_1..k_md), for the reverse call that
// reads abar next (fb(N) blocks).
template <typename T>
__global__ __launch_bounds__(BLOCK) void k_modadd_adj(size_t N, const cplx<T>* __restrict__ ub, const cplx<T>* __restrict__ a,
                                                      const cplx<T>* __restrict__ car, cplx<T>* __restrict__ abar,
                                                      double* __restrict__ thbar, VecSet<T> Kd, int md,
                                                      double* __restrict__ partials) {
    double acc[2 * GMAX];
#pragma unroll
    for (int v = 0; v < 2 * GMAX; ++v) acc[v] = 0.0;
    for (size_t p = blockIdx.x * (size_t)BLOCK + threadIdx.x; p < N; p += (size_t)gridDim.x * BLOCK) {
        const cplx<T> e = car[p];
        const cplx<T> y = ub[p];
        const cplx<T> ab = conjg(e) * y;
        abar[p] = ab;
        dots_add(acc, Kd, md, p, ab);
        const cplx<T> ae = a[p] * e;
        // Im(conj(y) * ae)
        thbar[p] -= double(y.re) * double(ae.im) - double(y.im) * double(ae.re);
    }
    if (md > 0) reduce_store<2 * GMAX>(acc, 2 * md, partials);
}

// The reverse of one level-2 ADR step's demodulation b = (g - A u) e^{-i theta} and of the
// previous step's re-modulation (k_modadd_adj), in one pass:
// with rbar = e^{i theta} bbar (formed at the neighbours on the fly)
//   thbar += Im(conj(bbar) b),  gbar += rbar,  ubar -= A^H rbar,
// and, when an (the earlier step's ADR result) is given, for the updated ubar
//   abar = e^{-i theta} ubar,  thbar -= Im(conj(ubar) an e^{i theta}),
// with md > 0 the per-block partials of <k_q, abar>, q < md (Kd: k_1..k_md), for the
// reverse call that reads abar next (fb(N) blocks).
// Interior nodes only, except that abar is written everywhere (0 on the ring).
template <typename T>
__global__ __launch_bounds__(BLOCK) void k_adr_step_adj(Geom G, const T* __restrict__ n2,
                                                        const cplx<T>* __restrict__ bbar, const cplx<T>* __restrict__ b,
                                                        const cplx<T>* __restrict__ car, cplx<T>* __restrict__ ubar,
                                                        cplx<T>* __restrict__ gbar, double* __restrict__ thbar,
                                                        const cplx<T>* __restrict__ an, cplx<T>* __restrict__ abar,
                                                        VecSet<T> Kd, int md, double* __restrict__ partials) {
    const int nx = G.nx, ny = G.ny;
    const size_t N = (size_t)nx * ny;
    double acc[2 * GMAX];
#pragma unroll
    for (int v = 0; v < 2 * GMAX; ++v) acc[v] = 0.0;
    auto RB = [&](int i, int j) -> cplx<T> {
        if (i <= 0 || j <= 0 || i >= ny || j >= nx) return cplx<T>{};
        const size_t q = (size_t)i * nx + j;
        return car[q] * bbar[q];
    };
    for (size_t p = blockIdx.x * (size_t)BLOCK + threadIdx.x; p < N; p += (size_t)gridDim.x * BLOCK) {
        int i, j;
        rowcol(p, nx, i, j);
        if (i == 0 || j == 0) {
            if (an) abar[p] = cplx<T>{};
            continue;
        }
        const cplx<T> y = bbar[p], bv = b[p], e = car[p];
        double th = thbar[p] + (double(y.re) * double(bv.im) - double(y.im) * double(bv.re));
        const cplx<T> rc = e * y;
        gbar[p] = gbar[p] + rc;
        cplx<T> kap = kappa_at<T>(G, n2[p], i, j);
        kap.im = -kap.im;
        const cplx<T> nb = ((RB(i - 1, j) + RB(i + 1, j)) + RB(i, j - 1)) + RB(i, j + 1);
        const cplx<T> ah = T(G.inv_h2) * (T(4) * rc - nb) - kap * rc;
        const cplx<T> ub = ubar[p] - ah;
        ubar[p] = ub;
        if (an) {
            const cplx<T> ab = conjg(e) * ub;
            abar[p] = ab;
            dots_add(acc, Kd, md, p, ab);
            const cplx<T> ae = an[p] * e;
            th -= double(ub.re) * double(ae.im) - double(ub.im) * double(ae.re);
        }
        thbar[p] = th;
    }
    if (md > 0) reduce_store<2 * GMAX>(acc, 2 * md, partials);
}

// ------------------------------------------------------------------ ADR operator adjoint

// Row coefficients of M at an unknown (fx = phi_x, fy = phi_y): with g = 2 sigma k / (2h),
//   centre 4/h^2 + c0 - i g 2(|fx|+|fy|), west -1/h^2 + i g (fx+|fx|), east -1/h^2 - i g (fx-|fx|),
//   south -1/h^2 + i g (fy+|fy|), north -1/h^2 - i g (fy-|fy|).
// (M^H y)(i,j) = conj(centre_ij) y_ij + conj(west_{i,j+1}) y_{i,j+1} + conj(east_{i,j-1}) y_{i,j-1}
//              + conj(south_{i+1,j}) y_{i+1,j} + conj(north_{i-1,j}) y_{i-1,j}.
template <typename T>
__device__ __forceinline__ cplx<T> applyMH_at(const AdrGeom& A, const T* __restrict__ px, const T* __restrict__ py,
                                              const cplx<T>* __restrict__ c0, const cplx<T>* __restrict__ y, int i,
                                              int j) {
    const int n = A.nx;  // nodes per row
    const T g = T(A.two_sk * A.inv_2h), ih2 = T(A.inv_h2);
    const size_t p = (size_t)i * n + j;
    const T fx = px[p], fy = py[p];
    const T ax = fx < T(0) ? -fx : fx, ay = fy < T(0) ? -fy : fy;
    const cplx<T> cc = c0[p];
    // conj(centre) = (4/h^2 + c0.re, -c0.im + g 2(|fx|+|fy|))
    cplx<T> out = mk<T>(T(4) * ih2 + cc.re, -cc.im + g * (T(2) * (ax + ay))) * y[p];
    if (j + 1 < n) {  // row (i, j+1), its west coefficient; conj: (-1/h^2, -g (fx+|fx|))
        const size_t q = p + 1;
        const T f = px[q], a = f < T(0) ? -f : f;
        out = out + mk<T>(-ih2, -g * (f + a)) * y[q];
    }
    if (j - 1 >= 1) {  // row (i, j-1), its east coefficient; conj: (-1/h^2, +g (fx-|fx|))
        const size_t q = p - 1;
        const T f = px[q], a = f < T(0) ? -f : f;
        out = out + mk<T>(-ih2, g * (f - a)) * y[q];
    }
    if (i + 1 < A.ny) {  // row (i+1, j), its south coefficient
        const size_t q = p + n;
        const T f = py[q], a = f < T(0) ? -f : f;
        out = out + mk<T>(-ih2, -g * (f + a)) * y[q];
    }
    if (i - 1 >= 1) {  // row (i-1, j), its north coefficient
        const size_t q = p - n;
        const T f = py[q], a = f < T(0) ? -f : f;
        out = out + mk<T>(-ih2, g * (f - a)) * y[q];
    }
    return out;
}

// Coefficient cotangents at row (i,j) for y = M a with output cotangent yb:
//   pxbar += 2 sigma k Im(conj(yb) dU/dfx), dU/dfx = (2 sx a_c - (1+sx) a_w + (1-sx) a_e) / (2h),
//   likewise pybar with (s, n) neighbours; c0bar += conj(a_c) yb.  d|f|/df = sign(f), 0 at 0.
template <typename T>
__device__ __forceinline__ void coef_grad_at(const AdrGeom& A, const T* __restrict__ px, const T* __restrict__ py,
                                             const cplx<T>* __restrict__ a, cplx<T> yb, int i, int j,
                                             double* __restrict__ pxb, double* __restrict__ pyb,
                                             c128* __restrict__ c0b) {
    const int n = A.nx, ny = A.ny;
    const size_t p = (size_t)i * n + j;
    const T fx = px[p], fy = py[p];
    const T sx = fx > T(0) ? T(1) : (fx < T(0) ? T(-1) : T(0));
    const T sy = fy > T(0) ? T(1) : (fy < T(0) ? T(-1) : T(0));
    const cplx<T> ac = a[p];
    const cplx<T> aw = ldz(a, i, j - 1, n, ny), ae = ldz(a, i, j + 1, n, ny);
    const cplx<T> as = ldz(a, i - 1, j, n, ny), an = ldz(a, i + 1, j, n, ny);
    const cplx<T> dux = T(A.inv_2h) * (((T(2) * sx) * ac - (T(1) + sx) * aw) + (T(1) - sx) * ae);
    const cplx<T> duy = T(A.inv_2h) * (((T(2) * sy) * ac - (T(1) + sy) * as) + (T(1) - sy) * an);
    const double ybr = double(yb.re), ybi = double(yb.im);
    pxb[p] += A.two_sk * (ybr * double(dux.im) - ybi * double(dux.re));
    pyb[p] += A.two_sk * (ybr * double(duy.im) - ybi * double(duy.re));
    c128 cb = c0b[p];
    cb.re += double(ac.re) * ybr + double(ac.im) * ybi;
    cb.im += double(ac.re) * ybi - double(ac.im) * ybr;
    c0b[p] = cb;
}

// ------------------------------------------------------------------ GMRES record

// k1 = b - M x0 (x0 may be null); partial ||k1||^2.
template <typename T>
__global__ __launch_bounds__(BLOCK) void k_gr_r0(AdrGeom A, const T* __restrict__ px, const T* __restrict__ py,
                                                 const cplx<T>* __restrict__ c0, const cplx<T>* __restrict__ b,
                                                 const cplx<T>* __restrict__ x0, cplx<T>* __restrict__ k1,
                                                 double* partials) {
    const int n = A.nx;  // nodes per row
    const size_t N = (size_t)n * A.ny;
    double acc[2] = {0.0, 0.0};
    for (size_t p = blockIdx.x * (size_t)BLOCK + threadIdx.x; p < N; p += (size_t)gridDim.x * BLOCK) {
        int i, j;
        rowcol(p, n, i, j);
        cplx<T> v{};
        if (i > 0 && j > 0) {
            v = b[p];
            if (x0) v = v - applyM_at(A, px, py, c0, x0, i, j);
            acc[0] += double(v.re) * double(v.re) + double(v.im) * double(v.im);
        }
        k1[p] = v;
    }
    reduce_store<2>(acc, 2, partials);
}

// k_{jj+1} = M k_jj / tau (1-based jj), and partial <k_i, k_{jj+1}> for i = 1..jj+1.
template <typename T>
__global__ __launch_bounds__(BLOCK) void k_gr_chain(AdrGeom A, const T* __restrict__ px, const T* __restrict__ py,
                                                    const cplx<T>* __restrict__ c0, VecSet<T> Kv, int jj, double inv_tau,
                                                    cplx<T>* __restrict__ kout, double* partials) {
    const int n = A.nx;  // nodes per row
    const size_t N = (size_t)n * A.ny;
    double acc[2 * (GMAX + 1)];
#pragma unroll
    for (int v = 0; v < 2 * (GMAX + 1); ++v) acc[v] = 0.0;
    const cplx<T>* __restrict__ kin = Kv.v[jj - 1];
    for (size_t p = blockIdx.x * (size_t)BLOCK + threadIdx.x; p < N; p += (size_t)gridDim.x * BLOCK) {
        int i, j;
        rowcol(p, n, i, j);
        cplx<T> v{};
        if (i > 0 && j > 0) {
            v = T(inv_tau) * applyM_at(A, px, py, c0, kin, i, j);
#pragma unroll
            for (int q = 0; q < GMAX + 1; ++q) {
                if (q < jj) {
                    const cplx<T> kq = Kv.v[q][p];
                    acc[2 * q] += double(kq.re) * double(v.re) + double(kq.im) * double(v.im);
                    acc[2 * q + 1] += double(kq.re) * double(v.im) - double(kq.im) * double(v.re);
                } else if (q == jj) {
                    acc[2 * q] += double(v.re) * double(v.re) + double(v.im) * double(v.im);
                }
            }
        }
        kout[p] = v;
    }
    reduce_store<2 * (GMAX + 1)>(acc, 2 * (jj + 1), partials);
}

// Output vectors k_1..k_{m+1} of a recorded GMRES call.
template <typename T>
struct KvOut {
    cplx<T>* v[GMAX + 1];
};

// The record of one GMRES(M) call in one pass on overlapped tiles (the s-step tile
// machinery): k_1 = b - M x0 (X0; else b) and k_{j+1} = M k_j / tau, built on the tile and
// a ring of M (+1 with x0) nodes in LDS, stored at the tile's nodes, with this block's
// Gram partials of k_1..k_{M+1} in the layout k_gr_solve sums (entry e at
// partials[e * nblk + block]; the imaginary part of a diagonal entry is 0).  tau is a
// power of two, so scaling the unscaled powers by tau^-j is exact.  Ring nodes are not
// written (the tape keeps them 0).  Tile<M, X0, true, TT>::tiles(nx, ny) blocks.
template <typename T, int M, bool X0, int TT>
__global__ __launch_bounds__(BLOCK) void k_gr_tile(AdrGeom A, const T* __restrict__ px, const T* __restrict__ py,
                                                   const cplx<T>* __restrict__ c0, const cplx<T>* __restrict__ b,
                                                   const cplx<T>* __restrict__ x0, KvOut<T> kout, double inv_tau,
                                                   double* __restrict__ partials) {
    using Tg = Tile<M, X0, true, TT>;
    constexpr int NE = (M + 1) * (M + 2);
    __shared__ cplx<T> buf[2 * Tg::NR];
    __shared__ double red[(BLOCK / 64) * NE];
    __shared__ double sums[NE];
    double acc[NE];
#pragma unroll
    for (int q = 0; q < NE; ++q) acc[q] = 0.0;
    T sc[M + 1];
    sc[0] = T(1);
#pragma unroll
    for (int j = 1; j <= M; ++j) sc[j] = sc[j - 1] * T(inv_tau);
    int ti, tj;
    tile_index(Tg::per_side(A.nx), ti, tj);
    sstep_tile<T, M, X0, true, TT>(A, ti, tj, px, py, c0, b, x0, buf,
                                   [&](int, int gi, int gj, bool own, cplx<T>, const cplx<T>(&k)[M + 1]) {
        if (!own) return;
        const unsigned p = (unsigned)(gi * A.nx + gj);
        double kr[M + 1], ki[M + 1];
#pragma unroll
        for (int j = 0; j <= M; ++j) {
            const cplx<T> v = sc[j] * k[j];
            st_off(kout.v[j], p, v);
            kr[j] = double(v.re);
            ki[j] = double(v.im);
        }
#pragma unroll
        for (int c = 0; c <= M; ++c) {
#pragma unroll
            for (int q = 0; q < c; ++q) {
                acc[c * (c + 1) + 2 * q] += kr[q] * kr[c] + ki[q] * ki[c];
                acc[c * (c + 1) + 2 * q + 1] += kr[q] * ki[c] - ki[q] * kr[c];
            }
            acc[c * (c + 1) + 2 * c] += kr[c] * kr[c] + ki[c] * ki[c];
        }
    });
    block_sum<NE, BLOCK / 64>(acc, NE, red, sums);
    store_partials(sums, NE, partials);
}

// sum over blocks b < nblk of row[b] in one wavefront: each lane issues its loads in
// batches of 32 before adding them (fixed order), then the wavefront sum.
__device__ __forceinline__ double wave_row_sum(const double* __restrict__ row, int nblk) {
    constexpr int SB = 32;
    const int lane = threadIdx.x & 63;
    double acc = 0.0;
    for (int b0 = 0; b0 < nblk; b0 += 64 * SB) {
        double t[SB];
#pragma unroll
        for (int k = 0; k < SB; ++k) {
            const int b = b0 + k * 64 + lane;
            t[k] = b < nblk ? row[b] : 0.0;
        }
#pragma unroll
        for (int k = 0; k < SB; ++k) acc += t[k];
    }
    return wave_sum(acc);
}

// Sums the per-block Gram partials of one taped GMRES call (entry e of every block at
// partials[e * nblk + b], e < (m+1)(m+2): the entries of k_1 first, then those of each
// k_{j+1} with k_1..k_{j+1}, the layout of R->gram), one wavefront per entry in a fixed
// order, into R->gram, then solves the least squares of the call from that Gram matrix
// of k_1..k_{m+1} (one thread, on LDS copies): normalised Cholesky of W^H W; columns whose
// pivot falls below 1e-14 (an invariant Krylov space) are dropped, which reproduces the
// early exit of Arnoldi.  One block of FBLOCK threads.
__global__ __launch_bounds__(FBLOCK) void k_gr_solve(const double* __restrict__ partials, int nblk,
                                                     GRec* __restrict__ R, double tau) {
    constexpr int NE = (GMAX + 1) * (GMAX + 2);
    __shared__ double gs[NE];
    __shared__ double Lf[2 * GMAX * GMAX], cs[2 * GMAX], ds[GMAX];
    __shared__ int rank_s, zero_s;
    const int m = R->m, ne = (m + 1) * (m + 2);
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    for (int e = wv; e < ne; e += FBLOCK / 64) {
        const double acc = wave_row_sum(partials + (size_t)e * nblk, nblk);
        if (lane == 0) {
            gs[e] = acc;
            R->gram[e] = acc;
        }
    }
    for (int q = threadIdx.x; q < 2 * GMAX * GMAX; q += FBLOCK) Lf[q] = 0.0;
    __syncthreads();
    if (threadIdx.x == 0) {
        auto Gc = [&](int i, int j) -> c128 {  // <k_i, k_j>, 1-based
            if (i <= j) return c128{gs[gram_off(i, j)], gs[gram_off(i, j) + 1]};
            return c128{gs[gram_off(j, i)], -gs[gram_off(j, i) + 1]};
        };
        for (int a = 0; a < 2 * GMAX; ++a) cs[a] = 0.0;
        for (int a = 0; a < GMAX; ++a) ds[a] = 0.0;
        const double b2 = Gc(1, 1).re;
        const int zero = !(b2 > 0.0) || !isfinite(b2);
        int rank = 0;
        if (!zero) {
            double sc[GMAX];
            for (int a = 0; a < m; ++a) {
                const double dg = tau * tau * Gc(a + 2, a + 2).re;
                sc[a] = dg > 0.0 ? 1.0 / sqrt(dg) : 0.0;
                ds[a] = sc[a];
            }
            // normalised matrix G^_ab = s_a s_b tau^2 <k_{a+2}, k_{b+2}>, Cholesky row by row
            for (int a = 0; a < m; ++a) {
                if (sc[a] == 0.0) break;
                bool ok = true;
                for (int b = 0; b <= a; ++b) {
                    const c128 g = Gc(a + 2, b + 2);
                    double gr = sc[a] * sc[b] * tau * tau * g.re, gi = sc[a] * sc[b] * tau * tau * g.im;
                    for (int q = 0; q < b; ++q) {  // - L_aq conj(L_bq)
                        const double lr = Lf[2 * (a * GMAX + q)], li = Lf[2 * (a * GMAX + q) + 1];
                        const double mr = Lf[2 * (b * GMAX + q)], mi = Lf[2 * (b * GMAX + q) + 1];
                        gr -= lr * mr + li * mi;
                        gi -= li * mr - lr * mi;
                    }
                    if (b < a) {
                        const double d = Lf[2 * (b * GMAX + b)];
                        Lf[2 * (a * GMAX + b)] = gr / d;
                        Lf[2 * (a * GMAX + b) + 1] = gi / d;
                    } else if (!(gr > 1e-14)) {
                        ok = false;
                    } else {
                        Lf[2 * (a * GMAX + a)] = sqrt(gr);
                        Lf[2 * (a * GMAX + a) + 1] = 0.0;
                    }
                }
                if (!ok) break;
                rank = a + 1;
            }
            // rhs_a = s_a tau <k_{a+2}, k_1>;  L L^H y = rhs;  c_a = s_a y_a
            double yr[GMAX], yi[GMAX];
            for (int a = 0; a < rank; ++a) {
                const c128 g = Gc(a + 2, 1);
                double rr = sc[a] * tau * g.re, ri = sc[a] * tau * g.im;
                for (int q = 0; q < a; ++q) {
                    const double lr = Lf[2 * (a * GMAX + q)], li = Lf[2 * (a * GMAX + q) + 1];
                    rr -= lr * yr[q] - li * yi[q];
                    ri -= lr * yi[q] + li * yr[q];
                }
                const double d = Lf[2 * (a * GMAX + a)];
                yr[a] = rr / d;
                yi[a] = ri / d;
            }
            for (int a = rank - 1; a >= 0; --a) {
                double rr = yr[a], ri = yi[a];
                for (int q = a + 1; q < rank; ++q) {  // - conj(L_qa) y_q
                    const double lr = Lf[2 * (q * GMAX + a)], li = Lf[2 * (q * GMAX + a) + 1];
                    rr -= lr * yr[q] + li * yi[q];
                    ri -= lr * yi[q] - li * yr[q];
                }
                const double d = Lf[2 * (a * GMAX + a)];
                yr[a] = rr / d;
                yi[a] = ri / d;
            }
            for (int a = 0; a < rank; ++a) {
                cs[2 * a] = sc[a] * yr[a];
                cs[2 * a + 1] = sc[a] * yi[a];
            }
        }
        rank_s = rank;
        zero_s = zero;
    }
    __syncthreads();
    for (int q = threadIdx.x; q < 2 * GMAX * GMAX; q += FBLOCK) R->Lf[q] = Lf[q];
    for (int q = threadIdx.x; q < 2 * GMAX; q += FBLOCK) {
        R->c[q] = cs[q];
        R->z[q] = 0.0;
    }
    for (int q = threadIdx.x; q < GMAX; q += FBLOCK) R->dsc[q] = ds[q];
    if (threadIdx.x == 0) {
        R->rank = rank_s;
        R->zero = zero_s;
    }
}

// Sums rows e = wv, wv + NW, ... (e < ne) of partials (nblk entries each) with one
// wavefront per row, the loads of a wavefront's rows issued together (SB per lane and row
// at a time); row sums to out[e].
template <int NEMAX, int THREADS, int SB>
__device__ __forceinline__ void rows_sum_sb(const double* __restrict__ partials, int nblk, int ne, double* out) {
    constexpr int NW = THREADS / 64, R = (NEMAX + NW - 1) / NW;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    double acc[R];
#pragma unroll
    for (int r = 0; r < R; ++r) acc[r] = 0.0;
    for (int b0 = 0; b0 < nblk; b0 += 64 * SB) {
        double t[R][SB];
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int e = wv + r * NW;
#pragma unroll
            for (int k = 0; k < SB; ++k) {
                const int b = b0 + k * 64 + lane;
                t[r][k] = (e < ne && b < nblk) ? partials[(size_t)e * nblk + b] : 0.0;
            }
        }
#pragma unroll
        for (int r = 0; r < R; ++r)
#pragma unroll
            for (int k = 0; k < SB; ++k) acc[r] += t[r][k];
    }
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int e = wv + r * NW;
        const double v = wave_sum(acc[r]);
        if (lane == 0 && e < ne) out[e] = v;
    }
}

// rows_sum_sb with a batch that fits the row length: one round of loads up to 1024
// blocks, without issuing loads for blocks beyond the rows on the small levels.
template <int NEMAX, int THREADS>
__device__ __forceinline__ void rows_sum(const double* __restrict__ partials, int nblk, int ne, double* out) {
    constexpr int NW = THREADS / 64, R = (NEMAX + NW - 1) / NW, SB = 32 / R > 0 ? 32 / R : 1;
    if (nblk <= 64)
        rows_sum_sb<NEMAX, THREADS, 1>(partials, nblk, ne, out);
    else if (nblk <= 256 && SB > 4)
        rows_sum_sb<NEMAX, THREADS, 4>(partials, nblk, ne, out);
    else if (nblk > 64 * SB && nblk <= 1024)
        rows_sum_sb<NEMAX, THREADS, 16>(partials, nblk, ne, out);
    else
        rows_sum_sb<NEMAX, THREADS, SB>(partials, nblk, ne, out);
}

// k_gr_solve for a compile-time dimension MM: the same sums and the same least squares,
// with the serial part on registers (fully unrolled loops; the rank as a flag).  One
// block of SBLOCK threads (fewer than FBLOCK, so that the serial thread has the
// registers it needs).
constexpr int SBLOCK = 512;
template <int MM>
__global__ __launch_bounds__(SBLOCK) void k_gr_solve_m(const double* __restrict__ partials, int nblk,
                                                       GRec* __restrict__ R, double tau) {
    constexpr int NE = (MM + 1) * (MM + 2);
    __shared__ double gs[NE];
    // one wavefront for up to three rows: a fixed batch measured faster here than the
    // row-length dispatch of rows_sum
    rows_sum_sb<NE, SBLOCK, 32 / ((NE + SBLOCK / 64 - 1) / (SBLOCK / 64))>(partials, nblk, NE, gs);
    __syncthreads();
    if (threadIdx.x != 0) return;
    double G[NE];
#pragma unroll
    for (int e = 0; e < NE; ++e) {
        G[e] = gs[e];
        R->gram[e] = G[e];
    }
    auto Gc = [&](int i, int j) -> c128 {  // <k_i, k_j>, 1-based
        if (i <= j) return c128{G[2 * (j * (j - 1) / 2 + i - 1)], G[2 * (j * (j - 1) / 2 + i - 1) + 1]};
        return c128{G[2 * (i * (i - 1) / 2 + j - 1)], -G[2 * (i * (i - 1) / 2 + j - 1) + 1]};
    };
    double Lr[MM][MM], Li[MM][MM], sc[MM], cr[MM], ci[MM];
#pragma unroll
    for (int a = 0; a < MM; ++a) {
        sc[a] = cr[a] = ci[a] = 0.0;
#pragma unroll
        for (int b = 0; b < MM; ++b) Lr[a][b] = Li[a][b] = 0.0;
    }
    const double b2 = Gc(1, 1).re;
    const int zero = !(b2 > 0.0) || !isfinite(b2);
    int rank = 0;
    if (!zero) {
#pragma unroll
        for (int a = 0; a < MM; ++a) {
            const double dg = tau * tau * Gc(a + 2, a + 2).re;
            sc[a] = dg > 0.0 ? 1.0 / sqrt(dg) : 0.0;
        }
        bool live = true;
#pragma unroll
        for (int a = 0; a < MM; ++a) {
            if (live && sc[a] == 0.0) live = false;
            bool ok = live;
#pragma unroll
            for (int b = 0; b <= a; ++b) {
                if (!ok) continue;
                const c128 gv = Gc(a + 2, b + 2);
                double gr = sc[a] * sc[b] * tau * tau * gv.re, gi = sc[a] * sc[b] * tau * tau * gv.im;
#pragma unroll
                for (int q = 0; q < b; ++q) {  // - L_aq conj(L_bq)
                    gr -= Lr[a][q] * Lr[b][q] + Li[a][q] * Li[b][q];
                    gi -= Li[a][q] * Lr[b][q] - Lr[a][q] * Li[b][q];
                }
                if (b < a) {
                    Lr[a][b] = gr / Lr[b][b];
                    Li[a][b] = gi / Lr[b][b];
                } else if (!(gr > 1e-14)) {
                    ok = false;
                } else {
                    Lr[a][a] = sqrt(gr);
                    Li[a][a] = 0.0;
                }
            }
            if (live && !ok) {
                live = false;
#pragma unroll
                for (int b = 0; b < MM; ++b) Lr[a][b] = Li[a][b] = 0.0;
            }
            if (live) rank = a + 1;
        }
        // rhs_a = s_a tau <k_{a+2}, k_1>;  L L^H y = rhs;  c_a = s_a y_a
        double yr[MM], yi[MM];
#pragma unroll
        for (int a = 0; a < MM; ++a) {
            yr[a] = yi[a] = 0.0;
            if (a >= rank) continue;
            const c128 gv = Gc(a + 2, 1);
            double rr = sc[a] * tau * gv.re, ri = sc[a] * tau * gv.im;
#pragma unroll
            for (int q = 0; q < a; ++q) {
                rr -= Lr[a][q] * yr[q] - Li[a][q] * yi[q];
                ri -= Lr[a][q] * yi[q] + Li[a][q] * yr[q];
            }
            yr[a] = rr / Lr[a][a];
            yi[a] = ri / Lr[a][a];
        }
#pragma unroll
        for (int a = MM - 1; a >= 0; --a) {
            if (a >= rank) continue;
            double rr = yr[a], ri = yi[a];
#pragma unroll
            for (int q = a + 1; q < MM; ++q) {  // - conj(L_qa) y_q
                if (q >= rank) continue;
                rr -= Lr[q][a] * yr[q] + Li[q][a] * yi[q];
                ri -= Lr[q][a] * yi[q] - Li[q][a] * yr[q];
            }
            yr[a] = rr / Lr[a][a];
            yi[a] = ri / Lr[a][a];
        }
#pragma unroll
        for (int a = 0; a < MM; ++a) {
            if (a >= rank) continue;
            cr[a] = sc[a] * yr[a];
            ci[a] = sc[a] * yi[a];
        }
    }
#pragma unroll
    for (int a = 0; a < MM; ++a) {
#pragma unroll
        for (int b = 0; b < MM; ++b) {
            R->Lf[2 * (a * GMAX + b)] = Lr[a][b];
            R->Lf[2 * (a * GMAX + b) + 1] = Li[a][b];
        }
        R->c[2 * a] = cr[a];
        R->c[2 * a + 1] = ci[a];
        R->z[2 * a] = R->z[2 * a + 1] = 0.0;
        R->dsc[a] = sc[a];
    }
    R->rank = rank;
    R->zero = zero;
}

// x = x0 + sum_{j=1..m} c_j k_j  (x0 may be null; may alias x).
template <typename T>
__global__ __launch_bounds__(BLOCK) void k_gr_combine(size_t N, VecSet<T> Kv, int m, const GRec* __restrict__ R,
                                                      const cplx<T>* x0, cplx<T>* x) {
    __shared__ T cf[2 * GMAX];
    if (threadIdx.x < 2 * GMAX) cf[threadIdx.x] = T(R->c[threadIdx.x]);
    __syncthreads();
    for (size_t p = blockIdx.x * (size_t)BLOCK + threadIdx.x; p < N; p += (size_t)gridDim.x * BLOCK) {
        cplx<T> v = x0 ? x0[p] : cplx<T>{};
        for (int q = 0; q < m; ++q) v = v + mk<T>(cf[2 * q], cf[2 * q + 1]) * Kv.v[q][p];
        x[p] = v;
    }
}

// Coarse tiles of the fused combination passes below (small, so that the small ADR levels
// still give hundreds of blocks).
constexpr int GRC = 8;
__host__ __device__ inline int gr_rr_blocks(int nx, int ny) {
    return ((nx / 2 + GRC - 1) / GRC) * ((ny / 2 + GRC - 1) / GRC);
}

// The combination of a recorded call, x = x0 + sum_{j=1..m} c_j k_j on the level of nx x ny
// nodes (as k_gr_combine, x0 may be null), fused with its bilinear prolongation into the
// finer level: out = base + P x out of place on the 2 nx x 2 ny fine nodes (the ring copies
// base, as k_prolong_copy).  A block owns a coarse tile of GRC x GRC nodes: it forms x there
// and on one more row and column in LDS (0 off the unknowns, the prolongation's rule),
// writes x at its own nodes, then the fine nodes 2 I0 .. 2 I0 + 2 GRC - 1 in both directions.
// gr_rr_blocks(2 nx, 2 ny) blocks.
template <typename T>
__global__ __launch_bounds__(BLOCK) void k_gr_combine_pa(int nx, int ny, VecSet<T> Kv, int m,
                                                         const GRec* __restrict__ R, const cplx<T>* x0,
                                                         cplx<T>* __restrict__ x, const cplx<T>* __restrict__ base,
                                                         cplx<T>* __restrict__ out) {
    constexpr int XW = GRC + 1;
    __shared__ cplx<T> xs[XW * XW];
    __shared__ T cf[2 * GMAX];
    if (threadIdx.x < 2 * GMAX) cf[threadIdx.x] = T(R->c[threadIdx.x]);
    __syncthreads();
    const int ntx = (nx + GRC - 1) / GRC;
    const int b = xcd_remap(blockIdx.x, gridDim.x);
    const int I0 = (b / ntx) * GRC, J0 = (b % ntx) * GRC;
    for (int q = threadIdx.x; q < XW * XW; q += BLOCK) {
        const int I = I0 + q / XW, J = J0 + q % XW;
        cplx<T> v{};
        if (I < ny && J < nx) {
            const size_t p = (size_t)I * nx + J;
            v = x0 ? x0[p] : cplx<T>{};
            for (int jv = 0; jv < m; ++jv) v = v + mk<T>(cf[2 * jv], cf[2 * jv + 1]) * Kv.v[jv][p];
            if (q / XW < GRC && q % XW < GRC) x[p] = v;
        }
        xs[q] = (I <= 0 || J <= 0 || I >= ny || J >= nx) ? cplx<T>{} : v;
    }
    __syncthreads();
    const int fnx = 2 * nx, fny = 2 * ny;
    for (int q = threadIdx.x; q < 4 * GRC * GRC; q += BLOCK) {
        const int i = 2 * I0 + q / (2 * GRC), j = 2 * J0 + q % (2 * GRC);
        if (i >= fny || j >= fnx) continue;
        const size_t p = (size_t)i * fnx + j;
        cplx<T> v = base[p];
        if (i > 0 && j > 0) {
            const int a = (i >> 1) - I0, c = (j >> 1) - J0;
            auto e = [&](int da, int dc) { return xs[(a + da) * XW + c + dc]; };
            cplx<T> w;
            if (!(i & 1) && !(j & 1)) {
                w = e(0, 0);
            } else if ((i & 1) && !(j & 1)) {
                w = T(0.5) * (e(0, 0) + e(1, 0));
            } else if (!(i & 1) && (j & 1)) {
                w = T(0.5) * (e(0, 0) + e(0, 1));
            } else {
                w = T(0.25) * (((e(0, 0) + e(1, 0)) + e(0, 1)) + e(1, 1));
            }
            v = v + w;
        }
        out[p] = v;
    }
}

// The combination of a recorded pre-smoother call (x0 = 0) fused with the restriction of
// its residual: x = sum_{j=1..m} c_j k_j on every fine node and rc = R (b - M x) on the
// coarse grid, where b - M x = k_1 - tau sum_j c_j k_{j+1} (M k_j = tau k_{j+1}), so no
// stencil of M is needed.  A block owns a coarse tile of GRC x GRC nodes (small, so that
// the small ADR levels still give hundreds of blocks) and the fine nodes
// 2I0 .. 2I0 + 2 GRC - 1 in both directions (it writes x there, 0 on the ring);
// gr_rr_blocks(nx, ny) blocks.
template <typename T>
__global__ __launch_bounds__(BLOCK) void k_gr_combine_rr(int nx, int ny, VecSet<T> Kv, int m,
                                                         const GRec* __restrict__ R, double tau,
                                                         cplx<T>* __restrict__ x, cplx<T>* __restrict__ rc) {
    constexpr int FW = 2 * GRC + 1, FH = 2 * GRC + 1;
    __shared__ cplx<T> r[FH * FW];
    __shared__ T cf[4 * GMAX];  // c_j, then tau c_j
    if (threadIdx.x < 2 * GMAX) {
        const T cv = T(R->c[threadIdx.x]);
        cf[threadIdx.x] = cv;
        cf[2 * GMAX + threadIdx.x] = T(tau) * cv;
    }
    __syncthreads();
    const int ncx = nx / 2, ncy = ny / 2;
    const int ntx = (ncx + GRC - 1) / GRC;
    const int b = xcd_remap(blockIdx.x, gridDim.x);
    const int I0 = (b / ntx) * GRC, J0 = (b % ntx) * GRC;
    const int fi0 = 2 * I0 - 1, fj0 = 2 * J0 - 1;
    for (int q = threadIdx.x; q < FH * FW; q += BLOCK) {
        const int ri = q / FW, rj = q - ri * FW;
        const int fi = fi0 + ri, fj = fj0 + rj;
        cplx<T> v{}, xv{};
        if (fi >= 1 && fj >= 1 && fi < ny && fj < nx) {
            const size_t p = (size_t)fi * nx + fj;
            v = Kv.v[0][p];
            for (int jv = 0; jv < m; ++jv) {
                const cplx<T> kj = Kv.v[jv][p], kn = Kv.v[jv + 1][p];
                xv = xv + mk<T>(cf[2 * jv], cf[2 * jv + 1]) * kj;
                v = v - mk<T>(cf[2 * GMAX + 2 * jv], cf[2 * GMAX + 2 * jv + 1]) * kn;
            }
        }
        r[q] = v;
        if (ri >= 1 && rj >= 1 && fi < ny && fj < nx) x[(size_t)fi * nx + fj] = xv;
    }
    __syncthreads();
    for (int q = threadIdx.x; q < GRC * GRC; q += BLOCK) {
        const int ci = q / GRC, cj = q - ci * GRC;
        const int I = I0 + ci, J = J0 + cj;
        if (I >= ncy || J >= ncx) continue;
        cplx<T> v{};
        if (I > 0 && J > 0) {
            const int l = (2 * ci + 1) * FW + 2 * cj + 1;
            const cplx<T> c = r[l];
            const cplx<T> ud = ((r[l - FW] + r[l + FW]) + r[l - 1]) + r[l + 1];
            const cplx<T> dg = ((r[l - FW - 1] + r[l - FW + 1]) + r[l + FW - 1]) + r[l + FW + 1];
            v = T(1.0 / 16.0) * ((T(4) * c + T(2) * ud) + dg);
        }
        rc[(size_t)I * ncx + J] = v;
    }
}

// ------------------------------------------------------------------ GMRES reverse

// cbar = <k_j, xbar> summed from the per-block partials (dots_add; one wavefront per
// entry, fixed order) into R->cbar, then (one thread, on LDS copies of the record)
// z = (W^H W)^{-1} cbar and the coefficients of kbar_1..kbar_{m+1} over (xbar, k_1..k_{m+1}):
//   rho = r0 - W c = k_1 - tau sum c_j k_{j+1},   Wz = tau sum z_j k_{j+1},
//   kbar_1 = conj(c_1) xbar + Wz,
//   kbar_{j+1} = [j < m] conj(c_{j+1}) xbar + tau (conj(z_j) rho - conj(c_j) Wz),  j = 1..m
// (differential of the normal equations: dc = (W^H W)^{-1} (dW^H rho + W^H (dr0 - dW c))).
// One block of FBLOCK threads.
__global__ __launch_bounds__(FBLOCK) void k_ga_prep(const double* __restrict__ partials, int nblk,
                                                    GRec* __restrict__ R, double tau) {
    constexpr int NC = 2 * (GMAX + 1) * (GMAX + 2);
    __shared__ double cb[2 * GMAX], Lf[2 * GMAX * GMAX], cs[2 * GMAX], ds[GMAX], zs[2 * GMAX], co[NC];
    const int m = R->m, rank = R->rank, zero = R->zero;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    for (int e = wv; e < 2 * m; e += FBLOCK / 64) {
        const double acc = wave_row_sum(partials + (size_t)e * nblk, nblk);
        if (lane == 0) {
            cb[e] = acc;
            R->cbar[e] = acc;
        }
    }
    for (int q = threadIdx.x; q < 2 * GMAX * GMAX; q += FBLOCK) Lf[q] = R->Lf[q];
    for (int q = threadIdx.x; q < 2 * GMAX; q += FBLOCK) {
        cs[q] = R->c[q];
        zs[q] = 0.0;
    }
    for (int q = threadIdx.x; q < GMAX; q += FBLOCK) ds[q] = R->dsc[q];
    for (int q = threadIdx.x; q < NC; q += FBLOCK) co[q] = 0.0;
    __syncthreads();
    if (threadIdx.x == 0 && !zero) {
        double yr[GMAX], yi[GMAX];
        for (int a = 0; a < rank; ++a) {
            double rr = ds[a] * cb[2 * a], ri = ds[a] * cb[2 * a + 1];
            for (int q = 0; q < a; ++q) {
                const double lr = Lf[2 * (a * GMAX + q)], li = Lf[2 * (a * GMAX + q) + 1];
                rr -= lr * yr[q] - li * yi[q];
                ri -= lr * yi[q] + li * yr[q];
            }
            const double d = Lf[2 * (a * GMAX + a)];
            yr[a] = rr / d;
            yi[a] = ri / d;
        }
        for (int a = rank - 1; a >= 0; --a) {
            double rr = yr[a], ri = yi[a];
            for (int q = a + 1; q < rank; ++q) {
                const double lr = Lf[2 * (q * GMAX + a)], li = Lf[2 * (q * GMAX + a) + 1];
                rr -= lr * yr[q] + li * yi[q];
                ri -= lr * yi[q] - li * yr[q];
            }
            const double d = Lf[2 * (a * GMAX + a)];
            yr[a] = rr / d;
            yi[a] = ri / d;
        }
        for (int a = 0; a < rank; ++a) {
            zs[2 * a] = ds[a] * yr[a];
            zs[2 * a + 1] = ds[a] * yi[a];
        }
        // vectors over (xbar, k_1, ..., k_{m+1}) as complex coefficient lists
        c128 rho[GMAX + 2], wz[GMAX + 2];
        for (int q = 0; q < m + 2; ++q) rho[q] = wz[q] = c128{0.0, 0.0};
        rho[1] = c128{1.0, 0.0};
        for (int j = 1; j <= m; ++j) {
            rho[j + 1] = c128{-tau * cs[2 * (j - 1)], -tau * cs[2 * (j - 1) + 1]};
            wz[j + 1] = c128{tau * zs[2 * (j - 1)], tau * zs[2 * (j - 1) + 1]};
        }
        auto row = [&](int r) { return co + r * GCOEF_STRIDE; };
        {  // kbar_1
            double* o = row(0);
            o[0] = cs[0];
            o[1] = -cs[1];
            for (int q = 1; q < m + 2; ++q) {
                o[2 * q] += wz[q].re;
                o[2 * q + 1] += wz[q].im;
            }
        }
        for (int j = 1; j <= m; ++j) {
            double* o = row(j);
            if (j < m) {
                o[0] = cs[2 * j];
                o[1] = -cs[2 * j + 1];
            }
            const c128 zc = c128{tau * zs[2 * (j - 1)], -tau * zs[2 * (j - 1) + 1]};  // tau conj(z_j)
            const c128 cc = c128{tau * cs[2 * (j - 1)], -tau * cs[2 * (j - 1) + 1]};  // tau conj(c_j)
            for (int q = 1; q < m + 2; ++q) {
                const c128 a = zc * rho[q], b = cc * wz[q];
                o[2 * q] += a.re - b.re;
                o[2 * q + 1] += a.im - b.im;
            }
        }
    }
    __syncthreads();
    for (int q = threadIdx.x; q < NC; q += FBLOCK) R->coef[q] = co[q];
    for (int q = threadIdx.x; q < 2 * GMAX; q += FBLOCK) R->z[q] = zs[q];
    if (threadIdx.x == 0) {
        R->one[0] = 1.0;
        R->one[1] = 0.0;
    }
}

// k_ga_prep for a compile-time dimension MM: the same sums and coefficient rows, with
// the serial part on registers; writes rows 0..MM of R->coef over (xbar, k_1..k_{MM+1}).
// One block of SBLOCK threads.
template <int MM>
__global__ __launch_bounds__(SBLOCK) void k_ga_prep_m(const double* __restrict__ partials, int nblk,
                                                      GRec* __restrict__ R, double tau) {
    constexpr int NV = MM + 2;
    __shared__ double cb[2 * MM];
    rows_sum<2 * MM, SBLOCK>(partials, nblk, 2 * MM, cb);
    __syncthreads();
    if (threadIdx.x != 0) return;
    const int rank = R->rank, zero = R->zero;
    double Lr[MM][MM], Li[MM][MM], ds[MM], cs[2 * MM], zs[2 * MM], cbr[2 * MM];
#pragma unroll
    for (int a = 0; a < MM; ++a) {
#pragma unroll
        for (int b = 0; b < MM; ++b) {
            Lr[a][b] = R->Lf[2 * (a * GMAX + b)];
            Li[a][b] = R->Lf[2 * (a * GMAX + b) + 1];
        }
        ds[a] = R->dsc[a];
        cs[2 * a] = R->c[2 * a];
        cs[2 * a + 1] = R->c[2 * a + 1];
        cbr[2 * a] = cb[2 * a];
        cbr[2 * a + 1] = cb[2 * a + 1];
        zs[2 * a] = zs[2 * a + 1] = 0.0;
    }
#pragma unroll
    for (int e = 0; e < 2 * MM; ++e) R->cbar[e] = cbr[e];
    double co[MM + 1][2 * NV];
#pragma unroll
    for (int r = 0; r <= MM; ++r)
#pragma unroll
        for (int e = 0; e < 2 * NV; ++e) co[r][e] = 0.0;
    if (!zero) {
        double yr[MM], yi[MM];
#pragma unroll
        for (int a = 0; a < MM; ++a) {
            yr[a] = yi[a] = 0.0;
            if (a >= rank) continue;
            double rr = ds[a] * cbr[2 * a], ri = ds[a] * cbr[2 * a + 1];
#pragma unroll
            for (int q = 0; q < a; ++q) {
                rr -= Lr[a][q] * yr[q] - Li[a][q] * yi[q];
                ri -= Lr[a][q] * yi[q] + Li[a][q] * yr[q];
            }
            yr[a] = rr / Lr[a][a];
            yi[a] = ri / Lr[a][a];
        }
#pragma unroll
        for (int a = MM - 1; a >= 0; --a) {
            if (a >= rank) continue;
            double rr = yr[a], ri = yi[a];
#pragma unroll
            for (int q = a + 1; q < MM; ++q) {
                if (q >= rank) continue;
                rr -= Lr[q][a] * yr[q] + Li[q][a] * yi[q];
                ri -= Lr[q][a] * yi[q] - Li[q][a] * yr[q];
            }
            yr[a] = rr / Lr[a][a];
            yi[a] = ri / Lr[a][a];
        }
#pragma unroll
        for (int a = 0; a < MM; ++a) {
            if (a >= rank) continue;
            zs[2 * a] = ds[a] * yr[a];
            zs[2 * a + 1] = ds[a] * yi[a];
        }
        // vectors over (xbar, k_1, ..., k_{MM+1}) as complex coefficient lists
        c128 rho[NV], wz[NV];
#pragma unroll
        for (int q = 0; q < NV; ++q) rho[q] = wz[q] = c128{0.0, 0.0};
        rho[1] = c128{1.0, 0.0};
#pragma unroll
        for (int j = 1; j <= MM; ++j) {
            rho[j + 1] = c128{-tau * cs[2 * (j - 1)], -tau * cs[2 * (j - 1) + 1]};
            wz[j + 1] = c128{tau * zs[2 * (j - 1)], tau * zs[2 * (j - 1) + 1]};
        }
        co[0][0] = cs[0];  // kbar_1
        co[0][1] = -cs[1];
#pragma unroll
        for (int q = 1; q < NV; ++q) {
            co[0][2 * q] += wz[q].re;
            co[0][2 * q + 1] += wz[q].im;
        }
#pragma unroll
        for (int j = 1; j <= MM; ++j) {
            if (j < MM) {
                co[j][0] = cs[2 * j];
                co[j][1] = -cs[2 * j + 1];
            }
            const c128 zc = c128{tau * zs[2 * (j - 1)], -tau * zs[2 * (j - 1) + 1]};  // tau conj(z_j)
            const c128 cc = c128{tau * cs[2 * (j - 1)], -tau * cs[2 * (j - 1) + 1]};  // tau conj(c_j)
#pragma unroll
            for (int q = 1; q < NV; ++q) {
                const c128 a = zc * rho[q], b = cc * wz[q];
                co[j][2 * q] += a.re - b.re;
                co[j][2 * q + 1] += a.im - b.im;
            }
        }
    }
#pragma unroll
    for (int r = 0; r <= MM; ++r)
#pragma unroll
        for (int e = 0; e < 2 * NV; ++e) R->coef[r * GCOEF_STRIDE + e] = co[r][e];
#pragma unroll
    for (int e = 0; e < 2 * MM; ++e) R->z[e] = zs[e];
    R->one[0] = 1.0;
    R->one[1] = 0.0;
}

// out = sum_q coef_q V_q + mu M^H accin   (accin may be null), and, when a is given,
// the coefficient cotangents of y = M a with ybar = mu accin.  V_0 = xbar, V_q = k_q.
template <typename T>
__global__ __launch_bounds__(BLOCK) void k_ga_step(AdrGeom A, const T* __restrict__ px, const T* __restrict__ py,
                                                   const cplx<T>* __restrict__ c0, VecSet<T> V, int nv,
                                                   const double* __restrict__ coef, const cplx<T>* __restrict__ accin,
                                                   double mu, const cplx<T>* __restrict__ a, cplx<T>* __restrict__ out,
                                                   double* __restrict__ pxb, double* __restrict__ pyb,
                                                   c128* __restrict__ c0b) {
    __shared__ T cf[2 * (GMAX + 2)];
    if (threadIdx.x < 2 * (GMAX + 2)) cf[threadIdx.x] = threadIdx.x < 2 * nv ? T(coef[threadIdx.x]) : T(0);
    __syncthreads();
    const int n = A.nx;  // nodes per row
    const size_t N = (size_t)n * A.ny;
    for (size_t p = blockIdx.x * (size_t)BLOCK + threadIdx.x; p < N; p += (size_t)gridDim.x * BLOCK) {
        int i, j;
        rowcol(p, n, i, j);
        cplx<T> v{};
        if (i > 0 && j > 0) {
            for (int q = 0; q < nv; ++q) v = v + mk<T>(cf[2 * q], cf[2 * q + 1]) * V.v[q][p];
            if (accin) {
                v = v + T(mu) * applyMH_at(A, px, py, c0, accin, i, j);
                if (a) coef_grad_at(A, px, py, a, T(mu) * accin[p], i, j, pxb, pyb, c0b);
            }
        }
        out[p] = v;
    }
}

// The reverse of one recorded GMRES(M) call (the k_ga_step sequence of one call) in one
// pass on overlapped tiles.  V_0 = xbar, V_{q+1} = k_q (q = 0..M); coef: the rows of
// k_ga_prep.  On the tile and a ring of H = M (+1 with x0) nodes, with the cotangent y
// and the vector a of each step in LDS:
//   y = kbar_{M+1} = sum_q coef[M][q] V_q,
//   y <- sum_q coef[j-2][q] V_q + (1/tau) M^H y   for j = M+1 .. 2   (then y = kbar_1),
// with the coefficient cotangents of k_j = M k_{j-1} / tau (a = k_{j-1}, ybar = y / tau)
// summed per node in registers; bbar = y (add: bbar += y) at the tile's nodes; with x0,
// xbar0 = xbar - M^H y and the cotangents of M x0 (ybar = -y); finally one
// read-modify-write of pxb, pyb, c0b per node.  Values off the unknowns are 0, so each
// application spoils one more ring of the region and the tile's own values are exact.
// The ring of bbar and xbar0 is not written.  Tiles of TT x TT unknowns, one per block.
template <typename T, int M, bool X0, int TT>
__global__ __launch_bounds__(BLOCK) void k_ga_tile(AdrGeom A, const T* __restrict__ px, const T* __restrict__ py,
                                                   const cplx<T>* __restrict__ c0, VecSet<T> V,
                                                   const double* __restrict__ coef, double inv_tau,
                                                   const cplx<T>* __restrict__ x0, cplx<T>* __restrict__ bbar, int add,
                                                   cplx<T>* __restrict__ xbar0, double* __restrict__ pxb,
                                                   double* __restrict__ pyb, c128* __restrict__ c0b) {
    constexpr int NV = M + 2;
    constexpr int H = M + (X0 ? 1 : 0);
    constexpr int RW = TT + 2 * H, NR = RW * RW, NPT = (NR + BLOCK - 1) / BLOCK;
    __shared__ cplx<T> ys[2 * NR];  // cotangent of the step (double buffer)
    __shared__ cplx<T> as[2 * NR];  // a of the step (double buffer)
    __shared__ T fxs[NR], fys[NR];
    __shared__ T cf[2 * NV * (M + 1)];
    const int tid = threadIdx.x;
    for (int q = tid; q < 2 * NV * (M + 1); q += BLOCK) {
        const int r = q / (2 * NV), e = q - r * (2 * NV);
        cf[q] = T(coef[r * GCOEF_STRIDE + e]);
    }
    const int nx = A.nx, ny = A.ny;
    int ti, tj;
    tile_index((nx - 2) / TT + 1, ti, tj);
    const int i0 = 1 + ti * TT - H, j0 = 1 + tj * TT - H;  // region node (0, 0)
    const T g = T(A.inv_2h) * T(A.two_sk), ih2 = T(A.inv_h2);
    cplx<T> v[NV][NPT], cc[NPT], xo[NPT];
    T fx[NPT], fy[NPT];
    bool ok[NPT], inner[NPT], own[NPT];
    unsigned gp[NPT];
#pragma unroll
    for (int k = 0; k < NPT; ++k) {
        const int q = tid + k * BLOCK;
        const int ri = q / RW, rj = q - ri * RW;
        const int gi = i0 + ri, gj = j0 + rj;
        ok[k] = q < NR && gi >= 1 && gi <= ny - 1 && gj >= 1 && gj <= nx - 1;
        inner[k] = ok[k] && ri >= 1 && ri <= RW - 2 && rj >= 1 && rj <= RW - 2;
        own[k] = ok[k] && ri >= H && ri < H + TT && rj >= H && rj < H + TT;
        gp[k] = ok[k] ? (unsigned)(gi * nx + gj) : 0u;
#pragma unroll
        for (int iv = 0; iv < NV; ++iv) v[iv][k] = cplx<T>{};
        cc[k] = xo[k] = cplx<T>{};
        fx[k] = fy[k] = T(0);
        if (ok[k]) {
#pragma unroll
            for (int iv = 0; iv < NV; ++iv) v[iv][k] = ld_off(V.v[iv], gp[k]);
            fx[k] = ld_off(px, gp[k]);
            fy[k] = ld_off(py, gp[k]);
            cc[k] = ld_off(c0, gp[k]);
            if constexpr (X0) xo[k] = ld_off(x0, gp[k]);
        }
        if (q < NR) {
            fxs[q] = fx[k];
            fys[q] = fy[k];
        }
    }
    __syncthreads();
    auto lincomb = [&](int row, int k) {
        cplx<T> r{};
#pragma unroll
        for (int iv = 0; iv < NV; ++iv) r = r + mk<T>(cf[row * 2 * NV + 2 * iv], cf[row * 2 * NV + 2 * iv + 1]) * v[iv][k];
        return r;
    };
    // M^H y at region node q (thread slot k): the conjugated centre of the node and the
    // conjugated coefficients of its neighbours' rows towards it (0 off the unknowns).
    auto mh = [&](const cplx<T>* y, int k) {
        const int q = tid + k * BLOCK;
        const T ax = fabs(fx[k]), ay = fabs(fy[k]);
        const cplx<T> c = y[q], e = y[q + 1], w = y[q - 1], n = y[q + RW], sth = y[q - RW];
        const T fe = fxs[q + 1], fw = fxs[q - 1], fn = fys[q + RW], fs = fys[q - RW];
        const T gwe = -g * (fe + fabs(fe)), gew = g * (fw - fabs(fw));    // west coefficient of e, east of w
        const T gsn = -g * (fn + fabs(fn)), gns = g * (fs - fabs(fs));    // south coefficient of n, north of s
        const T cr = cc[k].re + T(4) * ih2, ci = -(cc[k].im - g * (T(2) * (ax + ay)));
        T re = cr * c.re - ci * c.im, im = cr * c.im + ci * c.re;
        re -= ih2 * (((e.re + w.re) + n.re) + sth.re);
        im -= ih2 * (((e.im + w.im) + n.im) + sth.im);
        re -= ((gwe * e.im + gew * w.im) + gsn * n.im) + gns * sth.im;
        im += ((gwe * e.re + gew * w.re) + gsn * n.re) + gns * sth.re;
        return mk<T>(re, im);
    };
    double gx[NPT], gy[NPT];
    c128 g0[NPT];
#pragma unroll
    for (int k = 0; k < NPT; ++k) {
        gx[k] = gy[k] = 0.0;
        g0[k] = c128{0.0, 0.0};
    }
    // coefficient cotangents of y = M a at own node slot k (a in LDS buffer ab), ybar yb
    auto grad = [&](const cplx<T>* ab, int k, cplx<T> yb) {
        const int q = tid + k * BLOCK;
        const T sx = fx[k] > T(0) ? T(1) : (fx[k] < T(0) ? T(-1) : T(0));
        const T sy = fy[k] > T(0) ? T(1) : (fy[k] < T(0) ? T(-1) : T(0));
        const cplx<T> ac = ab[q], aw = ab[q - 1], ae = ab[q + 1], asd = ab[q - RW], an = ab[q + RW];
        const cplx<T> dux = T(A.inv_2h) * (((T(2) * sx) * ac - (T(1) + sx) * aw) + (T(1) - sx) * ae);
        const cplx<T> duy = T(A.inv_2h) * (((T(2) * sy) * ac - (T(1) + sy) * asd) + (T(1) - sy) * an);
        const double ybr = double(yb.re), ybi = double(yb.im);
        gx[k] += A.two_sk * (ybr * double(dux.im) - ybi * double(dux.re));
        gy[k] += A.two_sk * (ybr * double(duy.im) - ybi * double(duy.re));
        g0[k].re += double(ac.re) * ybr + double(ac.im) * ybi;
        g0[k].im += double(ac.re) * ybi - double(ac.im) * ybr;
    };
    cplx<T> y[NPT];
#pragma unroll
    for (int k = 0; k < NPT; ++k) y[k] = ok[k] ? lincomb(M, k) : cplx<T>{};
    const T mu = T(inv_tau);
#pragma unroll
    for (int s = 0; s < M; ++s) {  // kbar_{j-1} from kbar_j, j = M + 1 - s; a = k_{j-1} = V_{M-s}
        cplx<T>* yb = ys + (s & 1) * NR;
        cplx<T>* ab = as + (s & 1) * NR;
#pragma unroll
        for (int k = 0; k < NPT; ++k) {
            const int q = tid + k * BLOCK;
            if (q < NR) {
                yb[q] = y[k];
                ab[q] = v[M - s][k];
            }
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < NPT; ++k) {
            cplx<T> nv{};
            if (inner[k]) {
                nv = lincomb(M - 1 - s, k) + mu * mh(yb, k);
                if (own[k]) grad(ab, k, mu * y[k]);
            }
            y[k] = nv;
        }
    }
    // bbar (= or +=) kbar_1 at the tile's nodes
#pragma unroll
    for (int k = 0; k < NPT; ++k)
        if (own[k]) st_off(bbar, gp[k], add ? ld_off((const cplx<T>*)bbar, gp[k]) + y[k] : y[k]);
    if constexpr (X0) {  // xbar0 = xbar - M^H kbar_1, cotangents of M x0 with ybar = -kbar_1
        cplx<T>* yb = ys + (M & 1) * NR;
        cplx<T>* ab = as + (M & 1) * NR;
#pragma unroll
        for (int k = 0; k < NPT; ++k) {
            const int q = tid + k * BLOCK;
            if (q < NR) {
                yb[q] = y[k];
                ab[q] = xo[k];
            }
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < NPT; ++k) {
            if (!own[k]) continue;
            st_off(xbar0, gp[k], v[0][k] - mh(yb, k));
            grad(ab, k, T(-1) * y[k]);
        }
    }
#pragma unroll
    for (int k = 0; k < NPT; ++k) {
        if (!own[k]) continue;
        pxb[gp[k]] += gx[k];
        pyb[gp[k]] += gy[k];
        c128 b0 = c0b[gp[k]];
        b0.re += g0[k].re;
        b0.im += g0[k].im;
        c0b[gp[k]] = b0;
    }
}

// Reverse of bc = R (b - M x1) given bcbar (coarse): with t = P bcbar / 4,
//   bbar += t, xbar -= M^H t, coefficient cotangents with ybar = -t, a = x1.  In place.
// With md > 0 also the per-block partials of <k_q, xbar>, q < md (Kd: k_1..k_md), the
// dots of the reverse call that reads xbar next.
template <typename T>
__global__ __launch_bounds__(BLOCK) void k_adr_rr_adj(AdrGeom A, const T* __restrict__ px, const T* __restrict__ py,
                                                      const cplx<T>* __restrict__ c0, const cplx<T>* __restrict__ bcbar,
                                                      const cplx<T>* __restrict__ x1, cplx<T>* __restrict__ xbar,
                                                      cplx<T>* __restrict__ bbar, double* __restrict__ pxb,
                                                      double* __restrict__ pyb, c128* __restrict__ c0b, VecSet<T> Kd,
                                                      int md, double* __restrict__ partials) {
    const int n = A.nx, ny = A.ny;  // n: nodes per row
    const size_t N = (size_t)n * ny;
    const T g = T(A.two_sk * A.inv_2h), ih2 = T(A.inv_h2);
    auto tq = [&](int a, int b) -> cplx<T> {
        if (a <= 0 || b <= 0 || a >= ny || b >= n) return cplx<T>{};
        return T(0.25) * prolong_at<T, T>(bcbar, n / 2, ny / 2, a, b);
    };
    double acc[2 * GMAX];
#pragma unroll
    for (int v = 0; v < 2 * GMAX; ++v) acc[v] = 0.0;
    for (size_t p = blockIdx.x * (size_t)BLOCK + threadIdx.x; p < N; p += (size_t)gridDim.x * BLOCK) {
        int i, j;
        rowcol(p, n, i, j);
        if (i == 0 || j == 0) continue;
        const cplx<T> t = tq(i, j);
        bbar[p] = bbar[p] + t;
        // M^H t with t evaluated at the neighbours (same gather as applyMH_at)
        const T fx = px[p], fy = py[p];
        const T ax = fx < T(0) ? -fx : fx, ay = fy < T(0) ? -fy : fy;
        const cplx<T> cc = c0[p];
        cplx<T> mh = mk<T>(T(4) * ih2 + cc.re, -cc.im + g * (T(2) * (ax + ay))) * t;
        if (j + 1 < n) {
            const T f = px[p + 1], af = f < T(0) ? -f : f;
            mh = mh + mk<T>(-ih2, -g * (f + af)) * tq(i, j + 1);
        }
        if (j - 1 >= 1) {
            const T f = px[p - 1], af = f < T(0) ? -f : f;
            mh = mh + mk<T>(-ih2, g * (f - af)) * tq(i, j - 1);
        }
        if (i + 1 < ny) {
            const T f = py[p + n], af = f < T(0) ? -f : f;
            mh = mh + mk<T>(-ih2, -g * (f + af)) * tq(i + 1, j);
        }
        if (i - 1 >= 1) {
            const T f = py[p - n], af = f < T(0) ? -f : f;
            mh = mh + mk<T>(-ih2, g * (f - af)) * tq(i - 1, j);
        }
        const cplx<T> xb = xbar[p] - mh;
        xbar[p] = xb;
        coef_grad_at(A, px, py, x1, T(-1) * t, i, j, pxb, pyb, c0b);
        dots_add(acc, Kd, md, p, xb);  // the dots of the next reverse call
    }
    if (md > 0) reduce_store<2 * GMAX>(acc, 2 * md, partials);
}

// ------------------------------------------------------------------ phase cotangent

// Cotangent of the fine phase from the cotangents of phi_x, phi_y, c0 on one ADR
// level (and of the carrier phase theta on level 2), added to the level-2 array
// phib2 (level node (i,j) -> level-2 node (i*s2, j*s2)).  Reverse of k_adr_coef:
//   Px = pxbar + 2 k^2 phi_x Re(c0bar), Py likewise, Lap-bar = -sigma k Im(c0bar),
// pulled back through the central / one-sided differences of the coefficients.
template <typename T>
__global__ __launch_bounds__(BLOCK) void k_phi_adj(int n, int ny, int s2, int n2row, double k, int sigma,
                                                   const T* __restrict__ px, const T* __restrict__ py,
                                                   const double* __restrict__ pxb, const double* __restrict__ pyb,
                                                   const c128* __restrict__ c0b, const double* __restrict__ thb,
                                                   double* __restrict__ phib2) {
    // the level has n nodes per row and ny rows, spacing h = 1 / max(n, ny); n2row: nodes
    // per row of level 2
    const size_t N = (size_t)n * ny;
    const double nm = double(n > ny ? n : ny);
    const double i2h = 0.5 * nm, ih = nm, ih2 = nm * nm;
    const double k2 = k * k, sk = double(sigma) * k;
    auto PX = [&](int a, int b) -> double {
        if (a <= 0 || b <= 0 || a >= ny || b >= n) return 0.0;
        const size_t q = (size_t)a * n + b;
        return pxb[q] + 2.0 * k2 * double(px[q]) * c0b[q].re;
    };
    auto PY = [&](int a, int b) -> double {
        if (a <= 0 || b <= 0 || a >= ny || b >= n) return 0.0;
        const size_t q = (size_t)a * n + b;
        return pyb[q] + 2.0 * k2 * double(py[q]) * c0b[q].re;
    };
    auto LB = [&](int a, int b) -> double {
        if (a <= 0 || b <= 0 || a >= ny || b >= n) return 0.0;
        return -sk * c0b[(size_t)a * n + b].im;
    };
    for (size_t p = blockIdx.x * (size_t)BLOCK + threadIdx.x; p < N; p += (size_t)gridDim.x * BLOCK) {
        int i, j;
        rowcol(p, n, i, j);
        double v = 0.0;
        // along x (rows i >= 1): derivative index q = j-1, j, j+1 and the edge q = n-1
        if (i >= 1) {
            if (j - 1 >= 1 && j - 1 <= n - 2) v += PX(i, j - 1) * i2h + LB(i, j - 1) * ih2;
            if (j + 1 >= 1 && j + 1 <= n - 2) v += -PX(i, j + 1) * i2h + LB(i, j + 1) * ih2;
            if (j >= 1 && j <= n - 2) v += -2.0 * LB(i, j) * ih2;
            if (j == n - 1) v += PX(i, n - 1) * ih + LB(i, n - 1) * ih2;
            if (j == n - 2) v += -PX(i, n - 1) * ih - 2.0 * LB(i, n - 1) * ih2;
            if (j == n - 3) v += LB(i, n - 1) * ih2;
        }
        // along y (columns j >= 1): the edge is row ny - 1
        if (j >= 1) {
            if (i - 1 >= 1 && i - 1 <= ny - 2) v += PY(i - 1, j) * i2h + LB(i - 1, j) * ih2;
            if (i + 1 >= 1 && i + 1 <= ny - 2) v += -PY(i + 1, j) * i2h + LB(i + 1, j) * ih2;
            if (i >= 1 && i <= ny - 2) v += -2.0 * LB(i, j) * ih2;
            if (i == ny - 1) v += PY(ny - 1, j) * ih + LB(ny - 1, j) * ih2;
            if (i == ny - 2) v += -PY(ny - 1, j) * ih - 2.0 * LB(ny - 1, j) * ih2;
            if (i == ny - 3) v += LB(ny - 1, j) * ih2;
        }
        if (thb) v += sk * thb[p];
        phib2[(size_t)i * s2 * n2row + (size_t)j * s2] += v;
    }
}

// Fine-grid phase cotangent: the level-2 lattice (even fine indices) carries phib2,
// every other node 0 (the phase enters only through its injection).
template <typename TO>
__global__ __launch_bounds__(BLOCK) void k_phi_out(int nf, int nfy, const double* __restrict__ phib2,
                                                   TO* __restrict__ out) {
    // nf nodes per row and nfy rows on the fine grid; level 2 has nf / 2 per row
    const size_t N = (size_t)nf * nfy;
    const int n2 = nf / 2;
    for (size_t p = blockIdx.x * (size_t)BLOCK + threadIdx.x; p < N; p += (size_t)gridDim.x * BLOCK) {
        int i, j;
        rowcol(p, nf, i, j);
        double v = 0.0;
        if (!(i & 1) && !(j & 1)) v = phib2[(size_t)(i >> 1) * n2 + (j >> 1)];
        out[p] = TO(v);
    }
}

// ------------------------------------------------------------------ loss

// r = g - A u in FP64 on the fine grid (g, u in precision T), partial ||r||^2.
template <typename T>
__global__ __launch_bounds__(BLOCK) void k_loss_resid(Geom G, const double* __restrict__ n2, const cplx<T>* __restrict__ g,
                                                      const cplx<T>* __restrict__ u, c128* __restrict__ r,
                                                      double* partials) {
    const int n = G.nx;  // nodes per row
    const size_t N = (size_t)n * G.ny;
    double acc[1] = {0.0};
    for (size_t p = blockIdx.x * (size_t)BLOCK + threadIdx.x; p < N; p += (size_t)gridDim.x * BLOCK) {
        int i, j;
        rowcol(p, n, i, j);
        c128 v{};
        if (i > 0 && j > 0) {
            auto U = [&](int a, int b) { return ccast<double>(ldz(u, a, b, n, G.ny)); };
            const c128 c = U(i, j);
            const c128 nb = ((U(i - 1, j) + U(i + 1, j)) + U(i, j - 1)) + U(i, j + 1);
            const c128 kap = kappa_at<double>(G, n2[p], i, j);
            const c128 au = G.inv_h2 * (4.0 * c - nb) - kap * c;
            v = ccast<double>(g[p]) - au;
            acc[0] += v.re * v.re + v.im * v.im;
        }
        r[p] = v;
    }
    reduce_store<1>(acc, 1, partials);
}

// gu = -2 A^H r  (the cotangent of u for L = ||g - A u||^2), cast to T.
template <typename T>
__global__ __launch_bounds__(BLOCK) void k_loss_grad(Geom G, const double* __restrict__ n2, const c128* __restrict__ r,
                                                     cplx<T>* __restrict__ gu) {
    const int n = G.nx;  // nodes per row
    const size_t N = (size_t)n * G.ny;
    for (size_t p = blockIdx.x * (size_t)BLOCK + threadIdx.x; p < N; p += (size_t)gridDim.x * BLOCK) {
        int i, j;
        rowcol(p, n, i, j);
        cplx<T> v{};
        if (i > 0 && j > 0) v = ccast<T>(-2.0 * applyA_at(G, n2, r, i, j, true));
        gu[p] = v;
    }
}

}  // namespace helm
