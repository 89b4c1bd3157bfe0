// Shared device/host definitions of the Wave-ADR HIP library.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

namespace helm {

// Interleaved complex number with the memory layout of torch.complex64/128.
template <typename T>
struct alignas(2 * sizeof(T)) cplx {
    T re, im;
};

template <typename T>
__host__ __device__ __forceinline__ cplx<T> mk(T a, T b) {
    return cplx<T>{a, b};
}
template <typename T>
__host__ __device__ __forceinline__ cplx<T> operator+(cplx<T> a, cplx<T> b) {
    return {a.re + b.re, a.im + b.im};
}
template <typename T>
__host__ __device__ __forceinline__ cplx<T> operator-(cplx<T> a, cplx<T> b) {
    return {a.re - b.re, a.im - b.im};
}
template <typename T>
__host__ __device__ __forceinline__ cplx<T> operator*(cplx<T> a, cplx<T> b) {
    return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
template <typename T>
__host__ __device__ __forceinline__ cplx<T> operator*(T s, cplx<T> a) {
    return {s * a.re, s * a.im};
}
template <typename T>
__host__ __device__ __forceinline__ cplx<T> conjg(cplx<T> a) {
    return {a.re, -a.im};
}
// a / b
template <typename T>
__host__ __device__ __forceinline__ cplx<T> cdiv(cplx<T> a, cplx<T> b) {
    T d = b.re * b.re + b.im * b.im;
    return {(a.re * b.re + a.im * b.im) / d, (a.im * b.re - a.re * b.im) / d};
}

__device__ __forceinline__ void sincos_t(float x, float* s, float* c) { sincosf(x, s, c); }
__device__ __forceinline__ void sincos_t(double x, double* s, double* c) { sincos(x, s, c); }

template <typename To, typename Ti>
__host__ __device__ __forceinline__ cplx<To> ccast(cplx<Ti> a) {
    return {static_cast<To>(a.re), static_cast<To>(a.im)};
}

using c64 = cplx<float>;
using c128 = cplx<double>;

// Geometry and coefficients of one level of the hierarchy.  A level has nx columns and
// ny rows of stored nodes (row-major, index i * nx + j, i the row (y), j the column (x));
// both are powers of two, equal on square domains.
//   nx, ny   nodes per row / per column on this level
//   s        stride of the level in fine-grid indices, 2^(l-1)
//   nfx, nfy fine-grid nodes per row / per column
//   W        sponge width in fine cells (ramp 1 - d/W evaluated as 1 - d * inv_W)
//   inv_h2   1/h^2 of the level (h = 2^(l-1) / max(nfx, nfy))
//   sig_shift  sigma times the relative shift s0 of the shifted equation
// kappa(i, j) = k2 * n2(i, j) * (1 + i * (sig_str * rho^2 + sig_shift)), rho from the indices.
struct Geom {
    int nx, ny;
    int s;
    int nfx, nfy;
    int W;
    double inv_W;    // 1 / W
    double inv_h2;
    double k2;
    double sig_str;
    double sig_shift;
};

template <typename T>
__device__ __forceinline__ T sponge_ramp(int t, int nf, T inv_W) {
    int d = t < nf - t ? t : nf - t;
    T r = T(1) - T(d) * inv_W;
    return r > T(0) ? r : T(0);
}

template <typename T>
__device__ __forceinline__ cplx<T> kappa_at(const Geom& G, T n2, int i, int j) {
    T ri = sponge_ramp<T>(i * G.s, G.nfy, T(G.inv_W));
    T rj = sponge_ramp<T>(j * G.s, G.nfx, T(G.inv_W));
    T rho = ri > rj ? ri : rj;
    T kr = T(G.k2) * n2;
    return {kr, kr * (T(G.sig_str) * (rho * rho) + T(G.sig_shift))};
}

// Row and column of the flat index p on a grid of nx nodes per row; nx is a power of two,
// so this is a shift and a mask instead of a 64-bit division.
__device__ __forceinline__ void rowcol(size_t p, int nx, int& i, int& j) {
    const int sh = __builtin_ctz((unsigned)nx);
    i = (int)(p >> sh);
    j = (int)(p & (size_t)(nx - 1));
}

// Workgroup b of nb is dispatched to XCD b mod 8 (round robin).  This renumbering gives
// each XCD a contiguous range of work items (the first nb mod 8 XCDs one more), so that
// neighbouring tiles or strips share one L2.
__device__ __forceinline__ int xcd_remap(int b, int nb) {
    const int q = nb >> 3, r = nb & 7, x = b & 7;
    return x * q + (x < r ? x : r) + (b >> 3);
}

// Load with the implicit zero ring at row ny and column nx (i, j >= 0 always holds for
// callers).
template <typename V>
__device__ __forceinline__ V ldz(const V* __restrict__ a, int i, int j, int nx, int ny) {
    if (i >= ny || j >= nx) return V{};
    return a[(size_t)i * nx + j];
}

// ------------------------------------------------------------------ batched launches
// One launch can serve several problems of the same shape: launched with gridDim.z =
// n, block (x, y, z) works on problem p[z], whose device arrays all sit p[z] * stride
// bytes after those of problem 0 (the problems of one batch class are laid out in one
// arena, region by region in the same order).  A kernel therefore shifts every pointer
// argument by off() before it touches memory.  A single problem: n = 1, p[0] = 0,
// stride = 0.  aux carries one integer per problem for the kernels that need one.
constexpr int BMAX = 64;
struct BatchIdx {
    long long stride;
    int n;
    int p[BMAX];
    int aux[BMAX];
    __device__ __forceinline__ size_t off() const { return (size_t)p[blockIdx.z] * (size_t)stride; }
    __device__ __forceinline__ int aux_here() const { return aux[blockIdx.z]; }
};

// A pointer moved by o bytes (null stays null); argument structs define bsh_one too.  The
// shift is pointer arithmetic on the argument itself, so the result stays based on it
// (the restrict qualification of kernel arguments keeps its meaning).
template <typename Q>
__device__ __forceinline__ Q bsh_one(size_t o, Q q) {
    return q ? (Q)((const char*)q + o) : q;
}
template <typename... Q>
__device__ __forceinline__ void bshift(size_t o, Q&... q) {
    ((q = bsh_one(o, q)), ...);
}

// Maximum Krylov dimension supported by the device-side least squares.
constexpr int MAXM = 24;

// Device-resident state of one GMRES/FGMRES instance (all FP64).
struct KrylovScal {
    double beta;                          // ||r0||
    double scale[MAXM + 1];               // v_i = scale[i] * V_i
    double zscale[MAXM + 1];              // FGMRES: factor of V_j in the preconditioner input of z_j
    double H[2 * (MAXM + 1) * MAXM];      // complex Hessenberg, H(i,j) at 2*(i + j*(MAXM+1))
    double dots[2 * (MAXM + 2)];          // results of the last reduction pass
    double y[2 * MAXM];                   // least-squares solution
    double R[2 * (MAXM + 1) * MAXM];      // working copy for the Givens QR
    double e[2 * (MAXM + 1)];             // rotated right-hand side
    int cols;                             // Arnoldi columns completed
    int done;                             // 1: no further Arnoldi work (solved, breakdown, zero rhs)
    int m;                                // requested Krylov dimension
    unsigned pad;
};


}  // namespace helm
