// ADR-correction kernels: coefficients, upwind ADR operator, demodulation and
// re-modulation with the carrier e^{+- i sigma k phi}, ADR residual/restriction.
#pragma once

#include "kernels_wave.hpp"

namespace helm {

// Geometry of one ADR level.
struct AdrGeom {
    int nx, ny;        // nodes per row / per column
    double inv_h2;
    double inv_2h;     // 1/(2h)
    double two_sk;     // 2 * sigma * k (the advection factor is -i * two_sk)
};

// The level-2 carrier e^{i sigma k phi} from the phase reduced to [-pi, pi]
// (Cody-Waite reduction with a two-part 2 pi) and its sine and cosine, in FP64.
template <typename T>
__device__ __forceinline__ cplx<T> adr_carrier(double phi, double k, int sigma) {
    const double P1 = 6.283185307179586, P2 = 2.4492935982947064e-16;
    const double a = double(sigma) * k * phi;
    const double q = rint(a / P1);
    double t = fma(-q, P1, a);
    t = fma(-q, P2, t);
    double sn, cs;
    sincos(t, &sn, &cs);
    return mk<T>(T(cs), T(sn));
}

// phi_x, phi_y and Lap phi at unknown (i, j) of a level of nx x ny nodes with spacing h
// from the values P(a, b) of a field: second-order central differences inside,
// first-order one-sided ones at the last unknown of each axis (the boundary node of the
// open edge is not stored).
template <typename F>
__device__ __forceinline__ void fd_phase_rule(const F& P, int i, int j, int nx, int ny, double h, double& px,
                                              double& py, double& lap) {
    double pxx, pyy;
    const double c = P(i, j);
    if (j <= nx - 2) {
        px = (P(i, j + 1) - P(i, j - 1)) / (2.0 * h);
        pxx = ((P(i, j + 1) - 2.0 * c) + P(i, j - 1)) / (h * h);
    } else {
        px = (c - P(i, j - 1)) / h;
        pxx = ((c - 2.0 * P(i, j - 1)) + P(i, j - 2)) / (h * h);
    }
    if (i <= ny - 2) {
        py = (P(i + 1, j) - P(i - 1, j)) / (2.0 * h);
        pyy = ((P(i + 1, j) - 2.0 * c) + P(i - 1, j)) / (h * h);
    } else {
        py = (c - P(i - 1, j)) / h;
        pyy = ((c - 2.0 * P(i - 1, j)) + P(i - 2, j)) / (h * h);
    }
    lap = pxx + pyy;
}

// Stores phi_x, phi_y and the reaction term of level node p = (i, j):
//   c0 = -i sigma k Lap(phi) + k^2 (phi_x^2 + phi_y^2 - n2) - i sigma k^2 n2 delta
template <typename T>
__device__ __forceinline__ void adr_coef_store(const Geom& G, const double* __restrict__ n2f, int i, int j,
                                               size_t p, double px, double py, double lap, double k, int sigma,
                                               double strength, T* __restrict__ px_out, T* __restrict__ py_out,
                                               cplx<T>* __restrict__ c0_out) {
    const int s = G.s;
    const double nn = n2f[(size_t)i * s * G.nfx + (size_t)j * s];
    const double ri = sponge_ramp<double>(i * s, G.nfy, G.inv_W), rj = sponge_ramp<double>(j * s, G.nfx, G.inv_W);
    const double rho = ri > rj ? ri : rj;
    const double delta = strength * rho * rho + double(sigma) * G.sig_shift;  // sponge plus shift
    const double k2 = k * k;
    const double re = k2 * ((px * px + py * py) - nn);
    const double im = -(double(sigma) * k) * lap - ((double(sigma) * k2) * nn) * delta;
    px_out[p] = T(px);
    py_out[p] = T(py);
    c0_out[p] = mk<T>(T(re), T(im));
}

// Phase derivatives and reaction term on one ADR level, computed in FP64 from the
// fine phase by injection (stride s) with the finite-difference rule above.
// car (level 2 only, may be null): the carrier.
template <typename T, typename TP>
__global__ __launch_bounds__(BLOCK) void k_adr_coef(Geom G, const double* __restrict__ n2f,
                                                    const TP* __restrict__ phi, double k, int sigma, double strength,
                                                    T* __restrict__ px_out, T* __restrict__ py_out,
                                                    cplx<T>* __restrict__ c0_out, cplx<T>* __restrict__ car_out) {
    const int nx = G.nx, ny = G.ny, s = G.s, nfx = G.nfx;
    const size_t N = (size_t)nx * ny;
    const double h = 1.0 / (nx > ny ? nx : ny);
    for (size_t p = blockIdx.x * (size_t)BLOCK + threadIdx.x; p < N; p += (size_t)gridDim.x * BLOCK) {
        int i, j;
        rowcol(p, nx, i, j);
        auto P = [&](int a, int b) -> double { return double(phi[(size_t)a * s * nfx + (size_t)b * s]); };
        if (car_out) car_out[p] = adr_carrier<T>(P(i, j), k, sigma);
        if (i == 0 || j == 0) {
            px_out[p] = T(0);
            py_out[p] = T(0);
            c0_out[p] = cplx<T>{};
            continue;
        }
        double px, py, lap;
        fd_phase_rule(P, i, j, nx, ny, h, px, py, lap);
        adr_coef_store<T>(G, n2f, i, j, p, px, py, lap, k, sigma, strength, px_out, py_out, c0_out);
    }
}

// Plane-wave phase nbar (cs x + sn y) at the fine nodes (nx x ny), x = j h, y = i h with
// h = 1 / max(nx, ny), in FP64 with the products and the sum rounded separately (no
// contraction).
__global__ __launch_bounds__(BLOCK) void k_ray_phase(int nx, int ny, double nbar, double cs, double sn,
                                                     double* __restrict__ phi) {
    const size_t N = (size_t)nx * ny;
    const double nm = double(nx > ny ? nx : ny);
    for (size_t p = blockIdx.x * (size_t)BLOCK + threadIdx.x; p < N; p += (size_t)gridDim.x * BLOCK) {
        int i, j;
        rowcol(p, nx, i, j);
        const double x = double(j) / nm, y = double(i) / nm;
        phi[p] = __dmul_rn(nbar, __dadd_rn(__dmul_rn(cs, x), __dmul_rn(sn, y)));
    }
}

// (M x)(i,j) = -Delta_h x - 2 i sigma k U_h[x] + c0 x   (x scaled by xs)
template <typename T>
__device__ __forceinline__ cplx<T> applyM_at(const AdrGeom& A, const T* __restrict__ px, const T* __restrict__ py,
                                             const cplx<T>* __restrict__ c0, const cplx<T>* __restrict__ x, int i,
                                             int j) {
    const int nx = A.nx, ny = A.ny;
    const size_t p = (size_t)i * nx + j;
    const cplx<T> c = x[p];
    const cplx<T> w = ldz(x, i, j - 1, nx, ny), e = ldz(x, i, j + 1, nx, ny);
    const cplx<T> s = ldz(x, i - 1, j, nx, ny), nn = ldz(x, i + 1, j, nx, ny);
    const T fx = px[p], fy = py[p];
    const T ax = fx < T(0) ? -fx : fx, ay = fy < T(0) ? -fy : fy;
    const cplx<T> lap = T(A.inv_h2) * (T(4) * c - (((s + nn) + w) + e));
    const cplx<T> U = T(A.inv_2h) * (((((T(2) * (ax + ay)) * c - (fx + ax) * w) + (fx - ax) * e) - (fy + ay) * s) +
                                    (fy - ay) * nn);
    // -2 i sigma k U = (two_sk * U.im, -two_sk * U.re)
    const cplx<T> adv = mk<T>(T(A.two_sk) * U.im, -T(A.two_sk) * U.re);
    return lap + (adv + c0[p] * c);
}

template <typename T>
__global__ __launch_bounds__(BLOCK) void k_adr_apply(AdrGeom A, const T* __restrict__ px, const T* __restrict__ py,
                                                     const cplx<T>* __restrict__ c0, const cplx<T>* __restrict__ x,
                                                     cplx<T>* __restrict__ y, BatchIdx bi) {
    bshift(bi.off(), px, py, c0, x, y);
    int j, i0;
    tile_origin(A.nx, j, i0);
    if (j >= A.nx) return;
    for (int r = 0; r < RPT; ++r) {
        const int i = i0 + r;
        if (i >= A.ny) break;
        cplx<T> v{};
        if (i > 0 && j > 0) v = applyM_at(A, px, py, c0, x, i, j);
        y[(size_t)i * A.nx + j] = v;
    }
}

template <typename T>
__device__ __forceinline__ cplx<T> adr_resid_at(const AdrGeom& A, const T* px, const T* py, const cplx<T>* c0,
                                                const cplx<T>* b, const cplx<T>* x, int i, int j) {
    cplx<T> bv = b[(size_t)i * A.nx + j];
    if (x == nullptr) return bv;
    return bv - applyM_at(A, px, py, c0, x, i, j);
}

template <typename T>
struct AdrRes {
    AdrGeom A;
    const T* px;
    const T* py;
    const cplx<T>* c0;
    const cplx<T>* b;
    const cplx<T>* x;
    __device__ cplx<T> operator()(int i, int j) const { return adr_resid_at(A, px, py, c0, b, x, i, j); }
};

// rc = R (b - M x) on the next ADR level (x == nullptr: x = 0); rr_blocks(A.nx, A.ny) blocks.
template <typename T>
__global__ __launch_bounds__(BLOCK) void k_adr_resid_restrict(AdrGeom A, const T* __restrict__ px,
                                                              const T* __restrict__ py, const cplx<T>* __restrict__ c0,
                                                              const cplx<T>* __restrict__ b,
                                                              const cplx<T>* __restrict__ x, cplx<T>* __restrict__ rc, BatchIdx bi) {
    bshift(bi.off(), px, py, c0, b, x, rc);
    restrict_tile<T, T>(A.nx, A.ny, AdrRes<T>{A, px, py, c0, b, x}, rc);
}

// r_hat = (g - A u) e^{-i theta}   (car = e^{i theta})
template <typename T>
__global__ __launch_bounds__(BLOCK) void k_adr_demod(Geom G, const T* __restrict__ n2, const cplx<T>* __restrict__ g,
                                                     const cplx<T>* __restrict__ u, const cplx<T>* __restrict__ car,
                                                     cplx<T>* __restrict__ rhat, BatchIdx bi) {
    bshift(bi.off(), n2, g, u, car, rhat);
    int j, i0;
    tile_origin(G.nx, j, i0);
    if (j >= G.nx) return;
    for (int rr = 0; rr < RPT; ++rr) {
        const int i = i0 + rr;
        if (i >= G.ny) break;
        cplx<T> v{};
        const size_t p = (size_t)i * G.nx + j;
        if (i > 0 && j > 0) {
            cplx<T> r = resid_at(G, n2, g, u, i, j);
            v = r * conjg(car[p]);
        }
        rhat[p] = v;
    }
}

// Two consecutive ADR steps' joint: uout = uin + a e^{i theta} (the re-modulation of one
// step, out of place) and, when bout is given, bout = (g - A uout) e^{-i theta} (the
// demodulated residual of the next), with uout at the four neighbours formed on the fly.
// Every node is written (0 on the ring).
template <typename T>
__global__ __launch_bounds__(BLOCK) void k_adr_modadd_demod(Geom G, const T* __restrict__ n2,
                                                            const cplx<T>* __restrict__ g,
                                                            const cplx<T>* __restrict__ uin,
                                                            const cplx<T>* __restrict__ a,
                                                            const cplx<T>* __restrict__ car, cplx<T>* __restrict__ uout,
                                                            cplx<T>* __restrict__ bout) {
    const int nx = G.nx, ny = G.ny;
    const size_t N = (size_t)nx * ny;
    auto U = [&](int i, int j) -> cplx<T> {
        if (i <= 0 || j <= 0 || i >= ny || j >= nx) return cplx<T>{};
        const size_t q = (size_t)i * nx + j;
        return uin[q] + a[q] * car[q];
    };
    for (size_t p = blockIdx.x * (size_t)BLOCK + threadIdx.x; p < N; p += (size_t)gridDim.x * BLOCK) {
        int i, j;
        rowcol(p, nx, i, j);
        const cplx<T> uc = U(i, j);
        uout[p] = uc;
        if (!bout) continue;
        cplx<T> v{};
        if (i > 0 && j > 0) {
            const cplx<T> nb = ((U(i - 1, j) + U(i + 1, j)) + U(i, j - 1)) + U(i, j + 1);
            const cplx<T> lap = T(G.inv_h2) * (T(4) * uc - nb);
            const cplx<T> kap = kappa_at<T>(G, n2[p], i, j);
            v = (g[p] - (lap - kap * uc)) * conjg(car[p]);
        }
        bout[p] = v;
    }
}

// u += a e^{+i theta}   (car = e^{i theta})
template <typename T>
__global__ __launch_bounds__(BLOCK) void k_adr_modadd(size_t N, const cplx<T>* __restrict__ a,
                                                      const cplx<T>* __restrict__ car, cplx<T>* __restrict__ u, BatchIdx bi) {
    bshift(bi.off(), a, car, u);
    for (size_t p = blockIdx.x * (size_t)BLOCK + threadIdx.x; p < N; p += (size_t)gridDim.x * BLOCK)
        u[p] = u[p] + a[p] * car[p];
}

}  // namespace helm
