// Wave-cycle kernels: Helmholtz operator, residual, full weighting, bilinear
// prolongation, damped Jacobi and the Chebyshev semi-iteration steps.
//
// Every kernel runs 256-thread blocks (64 x 4) over 64 x 16 tiles of one level;
// a thread owns RPT = 4 consecutive rows of one column, so a wavefront reads
// 64 consecutive complex values per row (coalesced).  Tiles are assigned so
// that the blocks one XCD receives (block ids congruent mod 8) form a
// contiguous band of tile rows, keeping vertical halo reuse inside one L2.
#pragma once

#include "reduce.hpp"

namespace helm {

constexpr int TX = 64;   // tile width (one wavefront)
constexpr int TWY = 4;   // wavefronts per block
constexpr int RPT = 4;   // rows per thread
constexpr int TY = TWY * RPT;

__host__ __device__ inline int tiles_of(int nx, int ny) { return ((nx + TX - 1) / TX) * ((ny + TY - 1) / TY); }

// Column j and first row i0 of this thread's strip (nx nodes per row).
__device__ __forceinline__ void tile_origin(int nx, int& j, int& i0) {
    const int ntx = (nx + TX - 1) / TX;
    const int nb = gridDim.x;
    int b = blockIdx.x;
    b = xcd_remap(b, nb);
    const int tx = b % ntx, ty = b / ntx;
    j = tx * TX + threadIdx.x;
    i0 = ty * TY + threadIdx.y * RPT;
}

// Reduction kernels run at most MAXRED blocks; each block owns a contiguous chunk
// of tiles [t0, t1) (XCD-aware block order as above).
__host__ __device__ inline int red_blocks(int nx, int ny) {
    return tiles_of(nx, ny) < MAXRED ? tiles_of(nx, ny) : MAXRED;
}

__device__ __forceinline__ void tile_chunk(int nx, int ny, int& t0, int& t1) {
    const int nt = tiles_of(nx, ny);
    const int nb = gridDim.x;
    int b = blockIdx.x;
    b = xcd_remap(b, nb);
    const int per = (nt + nb - 1) / nb;
    t0 = b * per;
    t1 = t0 + per < nt ? t0 + per : nt;
}

__device__ __forceinline__ void tile_xy(int nx, int t, int& j, int& i0) {
    const int ntx = (nx + TX - 1) / TX;
    j = (t % ntx) * TX + threadIdx.x;
    i0 = (t / ntx) * TY + threadIdx.y * RPT;
}

// a on this block's 64 x 16 tile and a ring of R nodes, staged for LDS (row-major, width
// TX + 2R; 0 off the unknowns): tile_fetch issues a thread's loads into registers and
// tile_store writes them, so that a kernel can issue the loads of all its tile fields
// before it waits for any (one memory round trip per block).
template <int R>
struct TileRing {
    static constexpr int W = TX + 2 * R, NR = (TY + 2 * R) * W, NQ = (NR + BLOCK - 1) / BLOCK;
};
template <int R, typename V>
__device__ __forceinline__ void tile_fetch(const V* __restrict__ a, int nx, int ny, int it, int jt,
                                           V (&v)[TileRing<R>::NQ]) {
    using TR = TileRing<R>;
    const int tid = threadIdx.x + threadIdx.y * TX;
#pragma unroll
    for (int k = 0; k < TR::NQ; ++k) {
        const int q = tid + k * BLOCK;
        const int ri = q / TR::W, rj = q - ri * TR::W;
        const int gi = it - R + ri, gj = jt - R + rj;
        v[k] = V{};
        if (q < TR::NR && gi >= 1 && gj >= 1 && gi < ny && gj < nx) v[k] = a[(size_t)gi * nx + gj];
    }
}
template <int R, typename V>
__device__ __forceinline__ void tile_store(const V (&v)[TileRing<R>::NQ], V* s) {
    using TR = TileRing<R>;
    const int tid = threadIdx.x + threadIdx.y * TX;
#pragma unroll
    for (int k = 0; k < TR::NQ; ++k) {
        const int q = tid + k * BLOCK;
        if (q < TR::NR) s[q] = v[k];
    }
}

template <typename T>
__device__ __forceinline__ cplx<T> lap_at(const cplx<T>* __restrict__ u, int i, int j, int nx, int ny, T inv_h2) {
    cplx<T> c = u[(size_t)i * nx + j];
    cplx<T> nb = ldz(u, i - 1, j, nx, ny) + ldz(u, i + 1, j, nx, ny) + ldz(u, i, j - 1, nx, ny) +
                 ldz(u, i, j + 1, nx, ny);
    return inv_h2 * (T(4) * c - nb);
}

// (A u)(i,j) = -Delta_h u - kappa u ; conj_k selects A^* (conj(kappa)).
template <typename T>
__device__ __forceinline__ cplx<T> applyA_at(const Geom& G, const T* __restrict__ n2, const cplx<T>* __restrict__ u,
                                             int i, int j, bool conj_k) {
    const int nx = G.nx;
    cplx<T> kap = kappa_at<T>(G, n2[(size_t)i * nx + j], i, j);
    if (conj_k) kap.im = -kap.im;
    return lap_at(u, i, j, nx, G.ny, T(G.inv_h2)) - kap * u[(size_t)i * nx + j];
}

template <typename T>
__device__ __forceinline__ cplx<T> resid_at(const Geom& G, const T* __restrict__ n2, const cplx<T>* __restrict__ g,
                                            const cplx<T>* __restrict__ u, int i, int j) {
    cplx<T> gv = g[(size_t)i * G.nx + j];
    if (u == nullptr) return gv;
    return gv - applyA_at(G, n2, u, i, j, false);
}

// y = A x  (or A^* x)
template <typename T>
__global__ __launch_bounds__(BLOCK) void k_apply_A(Geom G, const T* __restrict__ n2, const cplx<T>* __restrict__ x,
                                                   cplx<T>* __restrict__ y, int conj_k, BatchIdx bi) {
    bshift(bi.off(), n2, x, y);
    int j, i0;
    tile_origin(G.nx, j, i0);
    if (j >= G.nx) return;
    for (int r = 0; r < RPT; ++r) {
        const int i = i0 + r;
        if (i >= G.ny) break;
        cplx<T> v{};
        if (i > 0 && j > 0) v = applyA_at(G, n2, x, i, j, conj_k != 0);
        y[(size_t)i * G.nx + j] = v;
    }
}

// r = g - A u   (u == nullptr means u = 0)
template <typename T>
__global__ __launch_bounds__(BLOCK) void k_residual(Geom G, const T* __restrict__ n2, const cplx<T>* __restrict__ g,
                                                    const cplx<T>* __restrict__ u, cplx<T>* __restrict__ r, BatchIdx bi) {
    bshift(bi.off(), n2, g, u, r);
    int j, i0;
    tile_origin(G.nx, j, i0);
    if (j >= G.nx) return;
    for (int rr = 0; rr < RPT; ++rr) {
        const int i = i0 + rr;
        if (i >= G.ny) break;
        cplx<T> v{};
        if (i > 0 && j > 0) v = resid_at(G, n2, g, u, i, j);
        r[(size_t)i * G.nx + j] = v;
    }
}

// Fine-grid FP64 residual with per-block partial sums of ||r||^2 and ||g||^2
// (finalized by k_finalize_sums).
__global__ __launch_bounds__(BLOCK) void k_residual_norms(Geom G, const double* __restrict__ n2,
                                                          const c128* __restrict__ g, const c128* __restrict__ u,
                                                          c128* __restrict__ r, double* partials, BatchIdx bi) {
    bshift(bi.off(), n2, g, u, r, partials);
    __shared__ double red[4 * 2];
    __shared__ double sums[2];
    double acc[2] = {0.0, 0.0};
    int t0, t1;
    tile_chunk(G.nx, G.ny, t0, t1);
    for (int t = t0; t < t1; ++t) {
        int j, i0;
        tile_xy(G.nx, t, j, i0);
        if (j >= G.nx) continue;
        for (int rr = 0; rr < RPT; ++rr) {
            const int i = i0 + rr;
            if (i >= G.ny) break;
            c128 v{};
            if (i > 0 && j > 0) {
                v = resid_at(G, n2, g, u, i, j);
                c128 gv = g[(size_t)i * G.nx + j];
                acc[0] += v.re * v.re + v.im * v.im;
                acc[1] += gv.re * gv.re + gv.im * gv.im;
            }
            if (r) r[(size_t)i * G.nx + j] = v;
        }
    }
    block_sum<2, 4>(acc, 2, red, sums);
    store_partials(sums, 2, partials);
}

// out[v] = sum over blocks of partials (one block of FBLOCK threads).
template <int K>
__global__ __launch_bounds__(FBLOCK) void k_finalize_sums(const double* __restrict__ partials, int nblk, int kcount,
                                                          double* out, BatchIdx bi) {
    bshift(bi.off(), partials, out);
    __shared__ double sums[K];
    final_sum<K>(partials, nblk, kcount, sums);
    if ((int)threadIdx.x < kcount) out[threadIdx.x] = sums[threadIdx.x];
}

// ------------------------------------------------------------------ residual + full weighting
// A block owns a coarse tile of RCX x RCY nodes: it evaluates the fine residual once
// on the (2 RCX + 1) x (2 RCY + 1) fine nodes around it into LDS, then applies the
// 9-point full weighting from LDS (each fine residual is computed about once
// instead of 2.25 times).  Coarse tiles are assigned XCD-aware as in tile_origin.
constexpr int RCX = 32, RCY = 16;

__host__ __device__ inline int rr_blocks(int nx, int ny) {
    const int ncx = nx / 2, ncy = ny / 2;
    return ((ncx + RCX - 1) / RCX) * ((ncy + RCY - 1) / RCY);
}

template <typename Tf, typename Tc, typename Res>
__device__ __forceinline__ void restrict_tile(int nx, int ny, const Res& res, cplx<Tc>* __restrict__ rc) {
    constexpr int FW = 2 * RCX + 1, FH = 2 * RCY + 1;
    __shared__ cplx<Tf> r[FH * FW];
    const int ncx = nx / 2, ncy = ny / 2;
    const int ntx = (ncx + RCX - 1) / RCX;
    const int nb = gridDim.x;
    int b = blockIdx.x;
    b = xcd_remap(b, nb);
    const int I0 = (b / ntx) * RCY, J0 = (b % ntx) * RCX;
    const int fi0 = 2 * I0 - 1, fj0 = 2 * J0 - 1;
    for (int q = threadIdx.x; q < FH * FW; q += BLOCK) {
        const int ri = q / FW, rj = q - ri * FW;
        const int fi = fi0 + ri, fj = fj0 + rj;
        cplx<Tf> v{};
        if (fi >= 1 && fj >= 1 && fi < ny && fj < nx) v = res(fi, fj);
        r[q] = v;
    }
    __syncthreads();
    for (int q = threadIdx.x; q < RCX * RCY; q += BLOCK) {
        const int ci = q / RCX, cj = q - ci * RCX;
        const int I = I0 + ci, J = J0 + cj;
        if (I >= ncy || J >= ncx) continue;
        cplx<Tf> v{};
        if (I > 0 && J > 0) {
            const int l = (2 * ci + 1) * FW + 2 * cj + 1;
            const cplx<Tf> c = r[l];
            const cplx<Tf> ud = ((r[l - FW] + r[l + FW]) + r[l - 1]) + r[l + 1];
            const cplx<Tf> dg = ((r[l - FW - 1] + r[l - FW + 1]) + r[l + FW - 1]) + r[l + FW + 1];
            v = Tf(1.0 / 16.0) * ((Tf(4) * c + Tf(2) * ud) + dg);
        }
        rc[(size_t)I * ncx + J] = ccast<Tc>(v);
    }
}

template <typename Tf>
struct HelmRes {
    Geom G;
    const Tf* n2;
    const cplx<Tf>* g;
    const cplx<Tf>* u;
    __device__ cplx<Tf> operator()(int i, int j) const { return resid_at(G, n2, g, u, i, j); }
};

// rc = R (g - A u) on the coarse grid of G.nx/2 x G.ny/2 nodes (u == nullptr: u = 0);
// rr_blocks(G.nx, G.ny) blocks.
template <typename Tf, typename Tc>
__global__ __launch_bounds__(BLOCK) void k_resid_restrict(Geom G, const Tf* __restrict__ n2,
                                                          const cplx<Tf>* __restrict__ g,
                                                          const cplx<Tf>* __restrict__ u, cplx<Tc>* __restrict__ rc, BatchIdx bi) {
    bshift(bi.off(), n2, g, u, rc);
    restrict_tile<Tf, Tc>(G.nx, G.ny, HelmRes<Tf>{G, n2, g, u}, rc);
}

// u += P ec (bilinear interpolation, P = 4 R^T); ec has ncx = nx/2 nodes per row and
// ncy = ny/2 rows.
template <typename Tc, typename Tf>
__device__ __forceinline__ cplx<Tf> prolong_at(const cplx<Tc>* __restrict__ ec, int ncx, int ncy, int i, int j) {
    const int I = i >> 1, J = j >> 1;
    auto e = [&](int a, int b) -> cplx<Tc> {
        if (a <= 0 || b <= 0 || a >= ncy || b >= ncx) return cplx<Tc>{};
        return ec[(size_t)a * ncx + b];
    };
    cplx<Tc> v;
    if (!(i & 1) && !(j & 1)) {
        v = e(I, J);
    } else if ((i & 1) && !(j & 1)) {
        v = Tc(0.5) * (e(I, J) + e(I + 1, J));
    } else if (!(i & 1) && (j & 1)) {
        v = Tc(0.5) * (e(I, J) + e(I, J + 1));
    } else {
        v = Tc(0.25) * (((e(I, J) + e(I + 1, J)) + e(I, J + 1)) + e(I + 1, J + 1));
    }
    return ccast<Tf>(v);
}

template <typename Tc, typename Tf>
__global__ __launch_bounds__(BLOCK) void k_prolong_add(int nx, int ny, const cplx<Tc>* __restrict__ ec,
                                                       cplx<Tf>* __restrict__ u, BatchIdx bi) {
    bshift(bi.off(), ec, u);
    int j, i0;
    tile_origin(nx, j, i0);
    if (j >= nx) return;
    for (int r = 0; r < RPT; ++r) {
        const int i = i0 + r;
        if (i >= ny) break;
        if (i == 0 || j == 0) continue;
        cplx<Tf>* p = u + (size_t)i * nx + j;
        *p = *p + prolong_at<Tc, Tf>(ec, nx / 2, ny / 2, i, j);
    }
}

// out = base + P ec out of place on every node (the ring copies base, which is 0 there).
template <typename T>
__global__ __launch_bounds__(BLOCK) void k_prolong_copy(int nx, int ny, const cplx<T>* __restrict__ ec,
                                                        const cplx<T>* __restrict__ base, cplx<T>* __restrict__ out) {
    int j, i0;
    tile_origin(nx, j, i0);
    if (j >= nx) return;
    for (int r = 0; r < RPT; ++r) {
        const int i = i0 + r;
        if (i >= ny) break;
        const size_t p = (size_t)i * nx + j;
        cplx<T> v = base[p];
        if (i > 0 && j > 0) v = v + prolong_at<T, T>(ec, nx / 2, ny / 2, i, j);
        out[p] = v;
    }
}

// u += P ec (assign: u = P ec) over pairs of fine columns (2J, 2J + 1): one coarse column
// pair and one row parity per thread, one 16-byte read-modify-write per pair in FP32.
// (ny - 1) (nx/2) pairs of rows 1..ny-1 (assign also writes row 0); coarse values off the
// unknowns read index 0 (the zero ring), so column 0 receives 0.
template <typename Tc, typename Tf>
__global__ __launch_bounds__(BLOCK) void k_prolong_pairs(int nx, int ny, const cplx<Tc>* __restrict__ ec,
                                                         cplx<Tf>* __restrict__ u, int assign, BatchIdx bi) {
    bshift(bi.off(), ec, u);
    const int ncx = nx / 2, ncy = ny / 2;
    const size_t NP = (size_t)ny * ncx;
    auto e = [&](int a, int b) -> cplx<Tc> {
        const bool in = a >= 1 && b >= 1 && a < ncy && b < ncx;
        return ec[in ? (size_t)a * ncx + b : 0];
    };
    for (size_t q = (size_t)blockIdx.x * BLOCK + threadIdx.x; q < NP; q += (size_t)gridDim.x * BLOCK) {
        int f, J;
        rowcol(q, ncx, f, J);
        const size_t p = (size_t)f * nx + 2 * J;
        cplx<Tf> ve{}, vo{};
        if (f > 0) {
            const int I = f >> 1;
            const cplx<Tc> e00 = e(I, J), e01 = e(I, J + 1);
            cplx<Tc> a, b;
            if (!(f & 1)) {
                a = e00;
                b = Tc(0.5) * (e00 + e01);
            } else {
                const cplx<Tc> e10 = e(I + 1, J), e11 = e(I + 1, J + 1);
                a = Tc(0.5) * (e00 + e10);
                b = Tc(0.25) * (((e00 + e10) + e01) + e11);
            }
            ve = ccast<Tf>(a);
            vo = ccast<Tf>(b);
        } else if (!assign) {
            continue;  // row 0 is the ring
        }
        if constexpr (sizeof(Tf) == 4) {
            float4* a4 = reinterpret_cast<float4*>(u + p);
            float4 w4 = assign ? make_float4(0.f, 0.f, 0.f, 0.f) : *a4;
            w4.x += ve.re;
            w4.y += ve.im;
            w4.z += vo.re;
            w4.w += vo.im;
            *a4 = w4;
        } else {
            u[p] = (assign ? cplx<Tf>{} : u[p]) + ve;
            u[p + 1] = (assign ? cplx<Tf>{} : u[p + 1]) + vo;
        }
    }
}

// uout = uin + w (g - A uin) / (4/h^2 - kappa)   (damped Jacobi, out of place)
template <typename T>
__global__ __launch_bounds__(BLOCK) void k_jacobi(Geom G, const T* __restrict__ n2, const cplx<T>* __restrict__ g,
                                                  const cplx<T>* __restrict__ uin, cplx<T>* __restrict__ uout,
                                                  const double* __restrict__ wp, BatchIdx bi) {
    bshift(bi.off(), n2, g, uin, uout, wp);
    const T w = T(wp[0]);
    int j, i0;
    tile_origin(G.nx, j, i0);
    if (j >= G.nx) return;
    for (int r = 0; r < RPT; ++r) {
        const int i = i0 + r;
        if (i >= G.ny) break;
        cplx<T> v{};
        if (i > 0 && j > 0) {
            const size_t p = (size_t)i * G.nx + j;
            cplx<T> kap = kappa_at<T>(G, n2[p], i, j);
            cplx<T> d = mk<T>(T(4) * T(G.inv_h2) - kap.re, -kap.im);
            cplx<T> res = resid_at(G, n2, g, uin, i, j);
            cplx<T> u0 = uin ? uin[p] : cplx<T>{};
            v = u0 + w * cdiv(res, d);
        }
        uout[(size_t)i * G.nx + j] = v;
    }
}

// Chebyshev start: r = A^* t, d = r / theta    (t = g - A u); cc[0] = 1 / theta of the
// level's coefficient table (a device array, one per problem).
template <typename T>
__global__ __launch_bounds__(BLOCK) void k_cheb_start(Geom G, const T* __restrict__ n2, const cplx<T>* __restrict__ t,
                                                      cplx<T>* __restrict__ r, cplx<T>* __restrict__ d,
                                                      const double* __restrict__ cc, BatchIdx bi) {
    bshift(bi.off(), n2, t, r, d, cc);
    const T inv_theta = T(cc[0]);
    int j, i0;
    tile_origin(G.nx, j, i0);
    if (j >= G.nx) return;
    for (int rr = 0; rr < RPT; ++rr) {
        const int i = i0 + rr;
        if (i >= G.ny) break;
        cplx<T> v{};
        if (i > 0 && j > 0) v = applyA_at(G, n2, t, i, j, true);
        const size_t p = (size_t)i * G.nx + j;
        r[p] = v;
        d[p] = inv_theta * v;
    }
}

// Chebyshev start from a nonzero u: t = g - A u on the 64 x 16 tile and a halo of one
// (in LDS, t is not stored), then r = A^* t and d = r / theta at the tile's nodes (cc[0] = 1/theta).
template <typename T>
__global__ __launch_bounds__(BLOCK) void k_cheb_start_res(Geom G, const T* __restrict__ n2,
                                                          const cplx<T>* __restrict__ g,
                                                          const cplx<T>* __restrict__ u, cplx<T>* __restrict__ r,
                                                          cplx<T>* __restrict__ d, const double* __restrict__ cc,
                                                          BatchIdx bi) {
    bshift(bi.off(), n2, g, u, r, d, cc);
    const T inv_theta = T(cc[0]);
    constexpr int UW = TX + 4, UH = TY + 4, HW = TX + 2, HH = TY + 2;
    __shared__ cplx<T> su[UH * UW];
    __shared__ cplx<T> sg[HH * HW];
    __shared__ T sn[HH * HW];
    __shared__ cplx<T> ts[HH * HW];
    const int nx = G.nx, ny = G.ny;
    const T ih2 = T(G.inv_h2);
    int j, i0;
    tile_origin(nx, j, i0);
    const int jt = j - (int)threadIdx.x, it = i0 - (int)threadIdx.y * RPT;  // tile origin
    const int tid = threadIdx.x + threadIdx.y * TX;
    cplx<T> fu[TileRing<2>::NQ], fg[TileRing<1>::NQ];
    T fn[TileRing<1>::NQ];
    tile_fetch<2>(u, nx, ny, it, jt, fu);
    tile_fetch<1>(g, nx, ny, it, jt, fg);
    tile_fetch<1>(n2, nx, ny, it, jt, fn);
    tile_store<2>(fu, su);
    tile_store<1>(fg, sg);
    tile_store<1>(fn, sn);
    __syncthreads();
    for (int q = tid; q < HH * HW; q += BLOCK) {  // t = g - A u on the tile and a ring of one
        const int ri = q / HW, rj = q - ri * HW;
        const int gi = it - 1 + ri, gj = jt - 1 + rj;
        cplx<T> v{};
        if (gi >= 1 && gj >= 1 && gi < ny && gj < nx) {
            const int l = (ri + 1) * UW + rj + 1;
            const cplx<T> c = su[l];
            const cplx<T> lap = ih2 * (T(4) * c - (((su[l - UW] + su[l + UW]) + su[l - 1]) + su[l + 1]));
            v = sg[q] - (lap - kappa_at<T>(G, sn[q], gi, gj) * c);
        }
        ts[q] = v;
    }
    __syncthreads();
    if (j >= nx) return;
    for (int rr = 0; rr < RPT; ++rr) {
        const int i = i0 + rr;
        if (i >= ny) break;
        const size_t p = (size_t)i * nx + j;
        cplx<T> v{};
        if (i > 0 && j > 0) {
            const int l = (i - it + 1) * HW + (j - jt + 1);
            cplx<T> kap = kappa_at<T>(G, sn[l], i, j);
            kap.im = -kap.im;
            const cplx<T> tc = ts[l];
            v = ih2 * (T(4) * tc - (((ts[l - HW] + ts[l + HW]) + ts[l - 1]) + ts[l + 1])) - kap * tc;
        }
        r[p] = v;
        d[p] = inv_theta * v;
    }
}

// Fused Chebyshev step on a 64 x 16 tile: t = A d_in on the tile and a halo of one
// (in LDS), then at the tile's nodes  u += d_in;  r -= A^* t;  d_out = c1 d_in + c2 r.
// d_in and d_out are different arrays (neighbouring tiles still read d_in).  c1 = cc[1],
// c2 = cc[2]: the row of this step in the level's coefficient table.
// mode bit 0 (CHEB_UZERO): u is zero on entry and is not read (its ring is written 0);
// bit 1 (CHEB_LAST): the iteration's final update u += d_out is done here as well, and
// r and d_out are not written (nothing reads them afterwards).
enum { CHEB_UZERO = 1, CHEB_LAST = 2 };
template <typename T>
__global__ __launch_bounds__(BLOCK) void k_cheb_fused(Geom G, const T* __restrict__ n2,
                                                      const cplx<T>* __restrict__ d_in, cplx<T>* __restrict__ d_out,
                                                      cplx<T>* __restrict__ r, cplx<T>* __restrict__ u,
                                                      const double* __restrict__ cc, int mode, BatchIdx bi) {
    bshift(bi.off(), n2, d_in, d_out, r, u, cc);
    const T c1 = T(cc[1]), c2 = T(cc[2]);
    constexpr int DW = TX + 4, DH = TY + 4, HW = TX + 2, HH = TY + 2;
    __shared__ cplx<T> sd[DH * DW];
    __shared__ T sn[HH * HW];
    __shared__ cplx<T> ts[HH * HW];
    const int nx = G.nx, ny = G.ny;
    const T ih2 = T(G.inv_h2);
    int j, i0;
    tile_origin(nx, j, i0);
    const int jt = j - (int)threadIdx.x, it = i0 - (int)threadIdx.y * RPT;  // tile origin
    const int tid = threadIdx.x + threadIdx.y * TX;
    // the tile fields and the own rows of r and u are all loaded before the first store
    cplx<T> fd[TileRing<2>::NQ];
    T fn[TileRing<1>::NQ];
    tile_fetch<2>(d_in, nx, ny, it, jt, fd);
    tile_fetch<1>(n2, nx, ny, it, jt, fn);
    cplx<T> rv0[RPT], uv0[RPT];
#pragma unroll
    for (int rr = 0; rr < RPT; ++rr) {
        const int i = i0 + rr;
        rv0[rr] = uv0[rr] = cplx<T>{};
        if (i >= 1 && i < ny && j >= 1 && j < nx) {
            const size_t p = (size_t)i * nx + j;
            rv0[rr] = r[p];
            if (!(mode & CHEB_UZERO)) uv0[rr] = u[p];
        }
    }
    tile_store<2>(fd, sd);
    tile_store<1>(fn, sn);
    __syncthreads();
    for (int q = tid; q < HH * HW; q += BLOCK) {  // t = A d_in on the tile and a ring of one
        const int ri = q / HW, rj = q - ri * HW;
        const int gi = it - 1 + ri, gj = jt - 1 + rj;
        cplx<T> v{};
        if (gi >= 1 && gj >= 1 && gi < ny && gj < nx) {
            const int l = (ri + 1) * DW + rj + 1;
            const cplx<T> c = sd[l];
            const cplx<T> lap = ih2 * (T(4) * c - (((sd[l - DW] + sd[l + DW]) + sd[l - 1]) + sd[l + 1]));
            v = lap - kappa_at<T>(G, sn[q], gi, gj) * c;
        }
        ts[q] = v;
    }
    __syncthreads();
    if (j >= nx) return;
    for (int rr = 0; rr < RPT; ++rr) {
        const int i = i0 + rr;
        if (i >= ny) break;
        const size_t p = (size_t)i * nx + j;
        if (i == 0 || j == 0) {  // keep the ring of the alternate d buffer (and of u) zero
            if (!(mode & CHEB_LAST)) d_out[p] = cplx<T>{};
            if (mode & CHEB_UZERO) u[p] = cplx<T>{};
            continue;
        }
        const int l = (i - it + 1) * HW + (j - jt + 1);
        cplx<T> kap = kappa_at<T>(G, sn[l], i, j);
        kap.im = -kap.im;
        const cplx<T> tc = ts[l];
        const cplx<T> aht = ih2 * (T(4) * tc - (((ts[l - HW] + ts[l + HW]) + ts[l - 1]) + ts[l + 1])) - kap * tc;
        const cplx<T> dv = sd[(i - it + 2) * DW + (j - jt + 2)];
        const cplx<T> rv = rv0[rr] - aht;
        const cplx<T> dn = c1 * dv + c2 * rv;
        const cplx<T> u1 = uv0[rr] + dv;
        if (mode & CHEB_LAST) {
            u[p] = u1 + dn;
        } else {
            u[p] = u1;
            r[p] = rv;
            d_out[p] = dn;
        }
    }
}

// ------------------------------------------------------------------ flat helpers
template <typename T>
__global__ __launch_bounds__(BLOCK) void k_axpy(size_t N, T a, const cplx<T>* __restrict__ x, cplx<T>* __restrict__ y, BatchIdx bi) {
    bshift(bi.off(), x, y);
    for (size_t p = blockIdx.x * (size_t)BLOCK + threadIdx.x; p < N; p += (size_t)gridDim.x * BLOCK) y[p] = y[p] + a * x[p];
}

template <typename To, typename Ti>
__global__ __launch_bounds__(BLOCK) void k_cast_scale(size_t N, const cplx<Ti>* __restrict__ x, cplx<To>* __restrict__ y,
                                                      double s, BatchIdx bi) {
    bshift(bi.off(), x, y);
    for (size_t p = blockIdx.x * (size_t)BLOCK + threadIdx.x; p < N; p += (size_t)gridDim.x * BLOCK) {
        cplx<Ti> v = x[p];
        y[p] = mk<To>(To(s * double(v.re)), To(s * double(v.im)));
    }
}

// y = (*s) cast(x) with the scale read from device memory
template <typename To, typename Ti>
__global__ __launch_bounds__(BLOCK) void k_cast_scale_dev(size_t N, const cplx<Ti>* __restrict__ x,
                                                          cplx<To>* __restrict__ y, const double* __restrict__ s, BatchIdx bi) {
    bshift(bi.off(), x, y, s);
    const double sc = *s;
    for (size_t p = blockIdx.x * (size_t)BLOCK + threadIdx.x; p < N; p += (size_t)gridDim.x * BLOCK) {
        cplx<Ti> v = x[p];
        y[p] = mk<To>(To(sc * double(v.re)), To(sc * double(v.im)));
    }
}

// y += s * cast(x)
template <typename To, typename Ti>
__global__ __launch_bounds__(BLOCK) void k_add_cast(size_t N, const cplx<Ti>* __restrict__ x, cplx<To>* __restrict__ y,
                                                    double s, BatchIdx bi) {
    bshift(bi.off(), x, y);
    for (size_t p = blockIdx.x * (size_t)BLOCK + threadIdx.x; p < N; p += (size_t)gridDim.x * BLOCK) {
        cplx<Ti> v = x[p];
        cplx<To> w = y[p];
        y[p] = mk<To>(To(double(w.re) + s * double(v.re)), To(double(w.im) + s * double(v.im)));
    }
}

// y += (*s) cast(x) with the scale read from device memory
template <typename To, typename Ti>
__global__ __launch_bounds__(BLOCK) void k_add_cast_dev(size_t N, const cplx<Ti>* __restrict__ x, cplx<To>* __restrict__ y,
                                                        const double* __restrict__ s, BatchIdx bi) {
    bshift(bi.off(), x, y, s);
    const double sc = *s;
    for (size_t p = blockIdx.x * (size_t)BLOCK + threadIdx.x; p < N; p += (size_t)gridDim.x * BLOCK) {
        cplx<Ti> v = x[p];
        cplx<To> w = y[p];
        y[p] = mk<To>(To(double(w.re) + sc * double(v.re)), To(double(w.im) + sc * double(v.im)));
    }
}

// From the squared norm sums[0] of a residual: sums[2] = 1 / ||r||, sums[3] = ||r||, with
// correctly rounded square root and division (the values the host computes).
__global__ void k_norm_scales(double* sums, BatchIdx bi) {
    bshift(bi.off(), sums);
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        const double rn = __dsqrt_rn(sums[0]);
        sums[2] = __ddiv_rn(1.0, rn);
        sums[3] = rn;
    }
}

template <typename T>
__global__ __launch_bounds__(BLOCK) void k_copy(size_t N, const cplx<T>* __restrict__ x, cplx<T>* __restrict__ y, BatchIdx bi) {
    bshift(bi.off(), x, y);
    for (size_t p = blockIdx.x * (size_t)BLOCK + threadIdx.x; p < N; p += (size_t)gridDim.x * BLOCK) y[p] = x[p];
}

template <typename T>
__global__ __launch_bounds__(BLOCK) void k_zero(size_t N, cplx<T>* __restrict__ y, BatchIdx bi) {
    bshift(bi.off(), y);
    for (size_t p = blockIdx.x * (size_t)BLOCK + threadIdx.x; p < N; p += (size_t)gridDim.x * BLOCK) y[p] = cplx<T>{};
}

// Injection of a fine real field (nfx nodes per row) to a level of nx x ny nodes
// (stride s); double -> T.
template <typename T, typename Ti>
__global__ __launch_bounds__(BLOCK) void k_inject_real(int nx, int ny, int s, int nfx, const Ti* __restrict__ fine,
                                                       T* __restrict__ out) {
    size_t N = (size_t)nx * ny;
    for (size_t p = blockIdx.x * (size_t)BLOCK + threadIdx.x; p < N; p += (size_t)gridDim.x * BLOCK) {
        int i, j;
        rowcol(p, nx, i, j);
        out[p] = T(fine[(size_t)i * s * nfx + (size_t)j * s]);
    }
}

// n2 = 1 / c^2 on the fine grid (FP64), with a check that c > 0 and finite.
__global__ __launch_bounds__(BLOCK) void k_slowness2(size_t N, const double* __restrict__ c, double* __restrict__ n2,
                                                     int* bad) {
    for (size_t p = blockIdx.x * (size_t)BLOCK + threadIdx.x; p < N; p += (size_t)gridDim.x * BLOCK) {
        double v = c[p];
        if (!(v > 0.0) || !isfinite(v)) {
            atomicOr(bad, 1);
            n2[p] = 0.0;
        } else {
            n2[p] = 1.0 / (v * v);
        }
    }
}

// Per-level statistics over the unknowns (1 <= i <= ny-1, 1 <= j <= nx-1): per-block
// max |4/h^2 - kappa|, max n2 and sum n2, stored as partials[3 * block + {0,1,2}]
// (combined on the host).
__global__ __launch_bounds__(BLOCK) void k_level_stats(Geom G, const double* __restrict__ n2, double* partials) {
    __shared__ double red[4 * 3];
    const int n = G.nx;
    const size_t N = (size_t)G.nx * G.ny;
    double mx = 0.0, mn2 = 0.0, sn2 = 0.0;
    for (size_t p = blockIdx.x * (size_t)BLOCK + threadIdx.x; p < N; p += (size_t)gridDim.x * BLOCK) {
        int i, j;
        rowcol(p, n, i, j);
        if (i == 0 || j == 0) continue;
        double v = n2[p];
        c128 kap = kappa_at<double>(G, v, i, j);
        double a = hypot(4.0 * G.inv_h2 - kap.re, kap.im);
        mx = a > mx ? a : mx;
        mn2 = v > mn2 ? v : mn2;
        sn2 += v;
    }
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    for (int off = 32; off > 0; off >>= 1) {
        double o1 = __shfl_xor(mx, off, 64), o2 = __shfl_xor(mn2, off, 64);
        mx = o1 > mx ? o1 : mx;
        mn2 = o2 > mn2 ? o2 : mn2;
        sn2 += __shfl_xor(sn2, off, 64);
    }
    if (lane == 0) {
        red[wave * 3 + 0] = mx;
        red[wave * 3 + 1] = mn2;
        red[wave * 3 + 2] = sn2;
    }
    __syncthreads();
    if (tid == 0) {
        double a = red[0], b = red[1], c = red[2];
        for (int w = 1; w < 4; ++w) {
            a = red[w * 3] > a ? red[w * 3] : a;
            b = red[w * 3 + 1] > b ? red[w * 3 + 1] : b;
            c += red[w * 3 + 2];
        }
        partials[blockIdx.x * 3 + 0] = a;
        partials[blockIdx.x * 3 + 1] = b;
        partials[blockIdx.x * 3 + 2] = c;
    }
}

}  // namespace helm
