// Travel-time phase on the device: the factored eikonal equation (Section 3.2.1).
//
// tau = tau0 tau1 with tau0 = |x - x0|, the exact solution for unit slowness
// (eq. eikonal_cons), and tau1 from |tau0 grad tau1 + tau1 grad tau0|^2 = s^2.
// Discretisation: the first-order Godunov upwind form on the fine nodes with grad tau0
// exact.  Per axis the neighbour of smaller tau is upwind; with sgn = +1 for the
// west/south one and -1 for the east/north one the discrete derivative of tau is
// a t - b with a = sgn r/h + g, b = sgn r tau1(q)/h (r = tau0, g = grad tau0,
// t = tau1 at the node).  Candidates: both axes ((a_x t - b_x)^2 + (a_y t - b_y)^2
// = s^2, larger root, kept if upwind on both axes), and each axis alone
// (sgn (a t - b) = s); the smallest one replaces tau1 if it is smaller.  Nodes
// within sqrt(2) h of the source are fixed at the straight-ray mean slowness.
//
// Fast sweeping: Gauss-Seidel passes in the four orders (i up, j up), (i up, j down),
// (i down, j up), (i down, j down).  A pass runs as a wavefront over B x B tiles
// (B = 64, or the shorter side when smaller; B divides both sides): the tiles of one
// anti-diagonal (in the pass's orientation) are independent
// and form one launch, one wavefront per tile; inside a tile the wavefront walks
// the node anti-diagonals with the tile and its one-node halo in LDS.  A node then
// sees exactly the values the sequential pass would give it (updated neighbours
// behind it, old ones ahead), so every pass equals the sequential one; the local
// update rounds every operation separately (no contraction; quotients by h = 2^-m
// are the exact products by 1/h), so the result is the same double precision numbers
// as a sequential implementation of the same steps.
#pragma once

#include "kernels_adr.hpp"

namespace helm {

struct EikSrc {
    int nx, ny;  // nodes per row / per column of the fine grid, h = 1 / max(nx, ny)
    double h, xs, ys;
    double rfix;  // nodes with r <= rfix are fixed
};

__device__ __forceinline__ double eik_r(const EikSrc& E, int i, int j) {
#pragma clang fp contract(off)
    const double dx = double(j) * E.h - E.xs;
    const double dy = double(i) * E.h - E.ys;
    return sqrt(dx * dx + dy * dy);
}

// New tau1 at global node (i, j) (not fixed, r = tau0 there, sp = s there) from the
// neighbour values tw, te, ts, tn (+inf where missing or not reached yet) and their
// tau0 values rw, re, rs, rn, or +inf when no candidate exists.  h = 1/max(nx, ny) is a
// power of two, so a quotient by h is the product by max(nx, ny), exactly.
__device__ __forceinline__ double eik_update(const EikSrc& E, int i, int j, double r, double sp, double tw,
                                             double te, double ts, double tn, double rw, double re, double rs,
                                             double rn) {
#pragma clang fp contract(off)
    const double inf = __builtin_huge_val();
    const double h = E.h, nh = double(E.nx > E.ny ? E.nx : E.ny);
    const double dx = double(j) * h - E.xs, dy = double(i) * h - E.ys;
    const double gx = dx / r, gy = dy / r;
    bool hx = false, hy = false;
    double tqx = inf, tqy = inf, ux = 0.0, uy = 0.0, sgx = 0.0, sgy = 0.0;
    if (tw < inf) {
        hx = true;
        tqx = rw * tw;
        ux = tw;
        sgx = 1.0;
    }
    if (te < inf) {
        const double v = re * te;
        if (!hx || v < tqx) {
            hx = true;
            tqx = v;
            ux = te;
            sgx = -1.0;
        }
    }
    if (ts < inf) {
        hy = true;
        tqy = rs * ts;
        uy = ts;
        sgy = 1.0;
    }
    if (tn < inf) {
        const double v = rn * tn;
        if (!hy || v < tqy) {
            hy = true;
            tqy = v;
            uy = tn;
            sgy = -1.0;
        }
    }
    double best = inf;
    const double s2 = sp * sp;
    const double ax = sgx * r * nh + gx, bx = sgx * r * ux * nh;
    const double ay = sgy * r * nh + gy, by = sgy * r * uy * nh;
    if (hx && hy) {
        const double A = ax * ax + ay * ay, B = ax * bx + ay * by, C = (bx * bx + by * by) - s2;
        if (A > 0.0) {
            const double disc = B * B - A * C;
            if (disc >= 0.0) {
                const double t = (B + sqrt(disc)) / A;
                if (sgx * (ax * t - bx) >= 0.0 && sgy * (ay * t - by) >= 0.0 && t < best) best = t;
            }
        }
    }
    if (hx && sgx * ax > 0.0) {
        const double t = (bx + sgx * sp) / ax;
        if (t < best) best = t;
    }
    if (hy && sgy * ay > 0.0) {
        const double t = (by + sgy * sp) / ay;
        if (t < best) best = t;
    }
    return best;
}

// s = sqrt(n^2) on the fine nodes.
__global__ __launch_bounds__(BLOCK) void k_eik_slowness(size_t N, const double* __restrict__ n2,
                                                        double* __restrict__ s) {
    for (size_t p = blockIdx.x * (size_t)BLOCK + threadIdx.x; p < N; p += (size_t)gridDim.x * BLOCK)
        s[p] = sqrt(n2[p]);
}

// tau1 = (s(node) + s(src node)) / 2 on the fixed nodes, +inf elsewhere.
__global__ __launch_bounds__(BLOCK) void k_eik_init(EikSrc E, const double* __restrict__ s, size_t psrc,
                                                    double* __restrict__ t1) {
    const size_t N = (size_t)E.nx * E.ny;
    const double ssrc = s[psrc];
    for (size_t p = blockIdx.x * (size_t)BLOCK + threadIdx.x; p < N; p += (size_t)gridDim.x * BLOCK) {
        int i, j;
        rowcol(p, E.nx, i, j);
        t1[p] = eik_r(E, i, j) <= E.rfix ? (s[p] + ssrc) / 2.0 : __builtin_huge_val();
    }
}

// One anti-diagonal d of B x B tiles of the pass (iup, jup): tile (I, J) of the
// pass's orientation (a = iup ? i : ny-1-i, b = jup ? j : nx-1-j) with I + J = d; B
// threads, B divides nx and ny.  part[tile] (tile in grid orientation, nx / B tiles per
// row) keeps the largest single decrease of tau1 in the round.
template <int B>
__global__ __launch_bounds__(B) void k_eik_pass(EikSrc E, const double* __restrict__ s, double* __restrict__ t1,
                                                int iup, int jup, int d, double* __restrict__ part) {
    constexpr int R = B + 2;
    __shared__ double tl[R * R];  // tau1 of the tile and its halo
    __shared__ double rl[R * R];  // tau0 there
    __shared__ double sl[B * B];
    __shared__ double red[B];
    const int n = E.nx, ny = E.ny, Tx = n / B, Ty = ny / B;
    const int I = (d < Tx ? 0 : d - Tx + 1) + (int)blockIdx.x, J = d - I;
    const int a0 = I * B, b0 = J * B;
    const int lane = threadIdx.x;
    const double inf = __builtin_huge_val();
    auto gi = [&](int a) { return iup ? a : ny - 1 - a; };
    auto gj = [&](int b) { return jup ? b : n - 1 - b; };
    for (int q = lane; q < R * R; q += B) {
        const int a = a0 - 1 + q / R, b = b0 - 1 + q % R;
        const bool in = a >= 0 && a < ny && b >= 0 && b < n;
        tl[q] = in ? t1[(size_t)gi(a) * n + gj(b)] : inf;
        rl[q] = in ? eik_r(E, gi(a), gj(b)) : 0.0;
    }
    for (int q = lane; q < B * B; q += B) sl[q] = s[(size_t)gi(a0 + q / B) * n + gj(b0 + q % B)];
    __syncthreads();
    // neighbours in grid orientation: west (j-1) is b-1 when jup, b+1 otherwise
    const int dw = jup ? -1 : 1, ds = iup ? -1 : 1;
    double dmax = 0.0;
    for (int k = 0; k < 2 * B - 1; ++k) {
        const int la = lane, lb = k - lane;
        if (lb >= 0 && lb < B) {
            const int i = gi(a0 + la), j = gj(b0 + lb);
            const int q = (la + 1) * R + (lb + 1);
            const double r = rl[q];
            if (r > E.rfix) {
                const double t = eik_update(E, i, j, r, sl[la * B + lb], tl[q + dw], tl[q - dw], tl[q + ds * R],
                                            tl[q - ds * R], rl[q + dw], rl[q - dw], rl[q + ds * R], rl[q - ds * R]);
                const double old = tl[q];
                if (t < old) {
                    const double dec = old == inf ? inf : old - t;
                    dmax = dec > dmax ? dec : dmax;
                    tl[q] = t;
                }
            }
        }
        __syncthreads();
    }
    for (int q = lane; q < B * B; q += B) t1[(size_t)gi(a0 + q / B) * n + gj(b0 + q % B)] = tl[(q / B + 1) * R + q % B + 1];
    red[lane] = dmax;
    __syncthreads();
    if (lane == 0) {
        double m = 0.0;
        for (int q = 0; q < B; ++q) m = red[q] > m ? red[q] : m;
        const int ti = iup ? I : Ty - 1 - I, tj = jup ? J : Tx - 1 - J;
        double* pp = part + (size_t)ti * Tx + tj;
        *pp = m > *pp ? m : *pp;
    }
}

// out[0] = max of x[0..N) and of 0 (one block of 1024 threads; maxima are exact in
// any order).
__global__ __launch_bounds__(1024) void k_eik_max(size_t N, const double* __restrict__ x, double* __restrict__ out) {
    __shared__ double sm[1024];
    double m = 0.0;
    for (size_t p = threadIdx.x; p < N; p += 1024) m = x[p] > m ? x[p] : m;
    sm[threadIdx.x] = m;
    __syncthreads();
    for (int w = 512; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) sm[threadIdx.x] = sm[threadIdx.x + w] > sm[threadIdx.x] ? sm[threadIdx.x + w] : sm[threadIdx.x];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = sm[0];
}

// phi = min(phi, tau0 tau1) (first arrival over the sources).
__global__ __launch_bounds__(BLOCK) void k_eik_phase(EikSrc E, const double* __restrict__ t1,
                                                     double* __restrict__ phi) {
    const size_t N = (size_t)E.nx * E.ny;
    for (size_t p = blockIdx.x * (size_t)BLOCK + threadIdx.x; p < N; p += (size_t)gridDim.x * BLOCK) {
        int i, j;
        rowcol(p, E.nx, i, j);
        const double v = eik_r(E, i, j) * t1[p];
        phi[p] = v < phi[p] ? v : phi[p];
    }
}

}  // namespace helm

namespace helm {

// ADR coefficients of one level from tau1 (fine, FP64) of the source (xs, ys) with the
// product rule of Section 3.2.1: with tau0 = r = |x - x0|, grad tau0 = (x - x0)/r and
// Lap tau0 = 1/r exact and the finite-difference rule applied to tau1,
//   grad phi = r grad tau1 + tau1 grad tau0,
//   Lap phi  = tau1 / r + 2 grad tau0 . grad tau1 + r Lap tau1;
// at nodes closer than one level spacing to the source the rule is applied to
// phi = r tau1 itself.  car (level 2 only, may be null): the carrier of phi.
template <typename T>
__global__ __launch_bounds__(BLOCK) void k_adr_coef_fac(Geom G, const double* __restrict__ n2f,
                                                        const double* __restrict__ tau1, double xs, double ys,
                                                        double k, int sigma, double strength,
                                                        T* __restrict__ px_out, T* __restrict__ py_out,
                                                        cplx<T>* __restrict__ c0_out, cplx<T>* __restrict__ car_out) {
    const int nx = G.nx, ny = G.ny, s = G.s, nfx = G.nfx;
    const size_t N = (size_t)nx * ny;
    const double h = 1.0 / (nx > ny ? nx : ny);
    auto R = [&](int a, int b) -> double {
        const double dx = double(b) * h - xs, dy = double(a) * h - ys;
        return sqrt(dx * dx + dy * dy);
    };
    auto T1 = [&](int a, int b) -> double { return tau1[(size_t)a * s * nfx + (size_t)b * s]; };
    auto PHI = [&](int a, int b) -> double { return R(a, b) * T1(a, b); };
    for (size_t p = blockIdx.x * (size_t)BLOCK + threadIdx.x; p < N; p += (size_t)gridDim.x * BLOCK) {
        int i, j;
        rowcol(p, nx, i, j);
        if (car_out) car_out[p] = adr_carrier<T>(PHI(i, j), k, sigma);
        if (i == 0 || j == 0) {
            px_out[p] = T(0);
            py_out[p] = T(0);
            c0_out[p] = cplx<T>{};
            continue;
        }
        double px, py, lap;
        const double r = R(i, j);
        if (r < h) {
            fd_phase_rule(PHI, i, j, nx, ny, h, px, py, lap);
        } else {
            double t1x, t1y, t1l;
            fd_phase_rule(T1, i, j, nx, ny, h, t1x, t1y, t1l);
            const double gx = (double(j) * h - xs) / r, gy = (double(i) * h - ys) / r;
            const double t1 = T1(i, j);
            px = r * t1x + t1 * gx;
            py = r * t1y + t1 * gy;
            lap = t1 / r + 2.0 * (gx * t1x + gy * t1y) + r * t1l;
        }
        adr_coef_store<T>(G, n2f, i, j, p, px, py, lap, k, sigma, strength, px_out, py_out, c0_out);
    }
}

}  // namespace helm
