// Level 1 from a zero iterate (the two fine-grid passes of the preconditioner
// application inside FGMRES).  One damped Jacobi sweep from u = 0 is pointwise,
// u0 = (w/d) g with d = 4/h^2 - kappa the diagonal of A.  Since d u0 = w g, the
// residual of u0 needs no kappa:
//   g - A u0 = (1 - w) g + h^-2 (sum of the four neighbours of u0),
// and the post-smoothing sweep from u = u0 + P ec folds to
//   u + (w/d)(g - A u) = (w/d) ((2 - w) g + h^-2 (sum of the neighbours of u)) + (1 - w) P ec.
// The two kernels use these forms and recompute u0 where they need it instead of
// storing it:
//   k_jac0_restrict:       rc = R (g - A u0)
//   k_jac0_prolong_jacobi: out = (w/d) ((2 - w) g + h^-2 sum_nb u) + (1 - w) P ec
// One wavefront owns a strip of 64 consecutive fine columns and walks down the rows of
// one segment, one fine row per step.  Lane l holds fine column c0 + l: west and east
// neighbours are lane shifts, the rows above and below sit in a register ring, and the
// loads run P rows ahead of their use.  The sponge ramp of the column is computed once
// per lane and that of the row once per step.  No LDS, no barrier; a strip's edge
// lanes are recomputed by its neighbours (2 of 64 columns), a segment's first rows
// by the segment above.
#pragma once

#include "kernels_sstep.hpp"

namespace helm {

// w / d at a node, d = 4/h^2 - kappa the diagonal of A; rho the sponge ramp there.
// FP32: one hardware reciprocal (relative error below 2^-22); FP64: a division.
template <typename T>
__device__ __forceinline__ cplx<T> jac_wd(const Geom& G, T n2v, T rho, T w) {
    const T kr = T(G.k2) * n2v;
    const T ki = kr * (T(G.sig_str) * (rho * rho) + T(G.sig_shift));
    const T dr = T(4) * T(G.inv_h2) - kr, di = -ki;
    T s;
    if constexpr (std::is_same<T, float>::value)
        s = w * __builtin_amdgcn_rcpf(dr * dr + di * di);
    else
        s = w / (dr * dr + di * di);
    return mk<T>(dr * s, -di * s);
}

constexpr int J0_W = 8;   // register ring (rows)
constexpr int J0R_CC = 30;  // coarse columns per strip of the restriction
constexpr int J0R_SC = 33;  // coarse rows per segment of the restriction (2 SC + 5 steps)
constexpr int J0P_CW = 62;  // fine columns per strip of the prolongation
constexpr int J0P_SR = 68;  // fine rows per segment of the prolongation (even; SR + 4 steps)
// Both marches run a fixed count of steps (a multiple of the ring), fully unrolled: a
// runtime loop would copy the ring registers at its back edge and wait there for every
// load in flight.  Steps past the segment compute rows that nothing stores.
constexpr int J0_STEPS = 72;
static_assert(2 * J0R_SC + 5 <= J0_STEPS && J0P_SR + 4 <= J0_STEPS && J0_STEPS % J0_W == 0, "march length");

__host__ __device__ inline int jac0r_units(int nx, int ny) {
    return ((nx / 2 + J0R_CC - 1) / J0R_CC) * ((ny / 2 + J0R_SC - 1) / J0R_SC);
}
__host__ __device__ inline int jac0p_units(int nx, int ny) {
    return ((nx - 2) / J0P_CW + 1) * ((ny - 2) / J0P_SR + 1);
}

// rc = R (g - A u0) on the coarse grid (nx/2 x ny/2, every coarse node written, the
// coarse ring with 0); jac0r_units(nx, ny) wavefronts of 64 threads.
template <typename Tf, typename Tc>
__global__ __launch_bounds__(64) void k_jac0_restrict(Geom G, const Tf* __restrict__ n2,
                                                        const cplx<Tf>* __restrict__ g,
                                                        const double* __restrict__ wp, cplx<Tc>* __restrict__ rc,
                                                        BatchIdx bi) {
    bshift(bi.off(), n2, g, wp, rc);
    // rows are loaded P ahead; a loaded row is still read one step after its own
    constexpr int W = J0_W, P = W - 2;
    const Tf w = Tf(wp[0]), w1 = Tf(1) - w, ih2 = Tf(G.inv_h2);
    const int nx = G.nx, ny = G.ny, ncx = nx / 2, ncy = ny / 2;
    const int lane = threadIdx.x;
    const int ns = (ncx + J0R_CC - 1) / J0R_CC;
    const int u = xcd_remap(blockIdx.x, gridDim.x);
    const int sg = u / ns, st = u - sg * ns;
    const int j = 2 * J0R_CC * st - 2 + lane;  // fine column of the lane
    const bool colok = j >= 1 && j <= nx - 1;
    const int jcl = colok ? j : 0;
    const Tf rj = sponge_ramp<Tf>(j * G.s, G.nfx, Tf(G.inv_W));
    const int Ib = sg * J0R_SC, Ie = (Ib + J0R_SC < ncy ? Ib + J0R_SC : ncy) - 1;
    const int J = j >> 1;
    const bool own = lane >= 2 && lane <= 61 && !(lane & 1) && J < ncx;
    const int q0 = 2 * Ib - 2;  // first fine row loaded
    cplx<Tf> gw[W], uw[W], rw[W];
    Tf nw[W];
    // every load is unconditional: off the unknowns it reads node 0 (the zero ring of g)
    auto load = [&](int q, cplx<Tf>& gv, Tf& nv) {
        const int qc = (q >= 1 && q <= ny - 1) ? q : 0;
        const unsigned p = (unsigned)(qc * nx + jcl);
        gv = ld_off(g, p);
        nv = ld_off(n2, p);
    };
#pragma unroll
    for (int s = 0; s < W; ++s) {
        gw[s] = uw[s] = rw[s] = cplx<Tf>{};
        nw[s] = Tf(0);
    }
    static_for<P>([&](auto pc) {
        constexpr int s = decltype(pc)::value;
        load(q0 + s, gw[s], nw[s]);
    });
#pragma unroll
    for (int t0 = 0; t0 < J0_STEPS; t0 += W) {
        static_for<W>([&](auto sc) {
            constexpr int s = decltype(sc)::value;
            constexpr int sm1 = (s + W - 1) % W, sm2 = (s + W - 2) % W, sm3 = (s + W - 3) % W, sp = (s + P) % W;
            const int q = q0 + t0 + s;
            load(q + P, gw[sp], nw[sp]);
            // u0 on row q (0 off the unknowns, where g was read as 0); no branch, so that
            // the loads ahead stay in flight
            const Tf ri = sponge_ramp<Tf>(q * G.s, G.nfy, Tf(G.inv_W));
            uw[s] = jac_wd<Tf>(G, nw[s], ri > rj ? ri : rj, w) * gw[s];
            // residual on row q - 1 (0 off the unknowns)
            const bool rok = q - 1 >= 1 && q - 1 <= ny - 1 && colok;
            const cplx<Tf> c = uw[sm1];
            const cplx<Tf> nb = ((uw[sm2] + uw[s]) + lane_prev(c)) + lane_next(c);
            const cplx<Tf> rv = w1 * gw[sm1] + ih2 * nb;
            rw[sm1] = mk<Tf>(rok ? rv.re : Tf(0), rok ? rv.im : Tf(0));
            // coarse row (q - 2) / 2 from the residual rows q - 3 .. q - 1
            const int qr = q - 2;
            if (!(qr & 1)) {
                const int I = qr >> 1;
                if (I >= Ib && I <= Ie) {
                    // (1/16)[1 2 1; 2 4 2; 1 2 1] as (1/4)[1 2 1] down the column, then across
                    const cplx<Tf> vs = (rw[sm3] + rw[sm1]) + Tf(2) * rw[sm2];
                    cplx<Tf> v = Tf(1.0 / 16.0) * ((lane_prev(vs) + lane_next(vs)) + Tf(2) * vs);
                    if (I == 0 || J == 0) v = cplx<Tf>{};
                    if (own) rc[(size_t)I * ncx + J] = ccast<Tc>(v);
                }
            }
        });
    }
}

// out = (w/d) ((2 - w) g + h^-2 sum_nb u) + (1 - w) P ec, u = u0 + P ec, on every fine
// node (0 on the ring); out must not overlap g.  jac0p_units(nx, ny) wavefronts of 64
// threads.
template <typename Tc, typename Tf>
__global__ __launch_bounds__(64) void k_jac0_prolong_jacobi(Geom G, const Tf* __restrict__ n2,
                                                              const cplx<Tf>* __restrict__ g,
                                                              const cplx<Tc>* __restrict__ ec,
                                                              const double* __restrict__ wp,
                                                              cplx<Tf>* __restrict__ out, BatchIdx bi) {
    bshift(bi.off(), n2, g, ec, wp, out);
    // rows are loaded P ahead; a loaded odd row's coarse values are read two steps after
    // its own
    constexpr int W = J0_W, P = W - 3;
    const Tf w = Tf(wp[0]), w1 = Tf(1) - w, w2 = Tf(2) - w, ih2 = Tf(G.inv_h2);
    const int nx = G.nx, ny = G.ny, ncx = nx / 2, ncy = ny / 2;
    const int lane = threadIdx.x;
    const int ns = (nx - 2) / J0P_CW + 1;
    const int u = xcd_remap(blockIdx.x, gridDim.x);
    const int sg = u / ns, st = u - sg * ns;
    const int j = J0P_CW * st + lane;  // fine column of the lane
    const bool colok = j >= 1 && j <= nx - 1;
    const int jcl = colok ? j : 0;
    const Tf rj = sponge_ramp<Tf>(j * G.s, G.nfx, Tf(G.inv_W));
    const bool own = ((lane >= 1 && lane <= J0P_CW) || j == 0) && j <= nx - 1;
    const int rb = 1 + sg * J0P_SR, re = (rb + J0P_SR - 1 < ny - 1 ? rb + J0P_SR - 1 : ny - 1);
    if (sg == 0 && own) out[j] = cplx<Tf>{};  // row 0
    // coarse columns of the lane: J and, for odd j, J + 1 (0 off the coarse unknowns)
    const int Jc = j >> 1;
    const bool jodd = j & 1;
    const int cJ0 = (Jc >= 1 && Jc < ncx) ? Jc : -1, cJ1 = (Jc + 1 >= 1 && Jc + 1 < ncx) ? Jc + 1 : -1;
    const int q0 = rb - 2;  // odd: the slot of every odd row q carries coarse row (q + 1) / 2
    cplx<Tf> gw[W], uw[W], wdw[W], pew[W];
    Tf nw[W];
    cplx<Tc> e0w[W], e1w[W];  // coarse row (q + 1) / 2 at J, J + 1 (odd slots)
    auto load = [&](int q, cplx<Tf>& gv, Tf& nv, cplx<Tc>& e0, cplx<Tc>& e1, bool odd) {
        const int qc = (q >= 1 && q <= ny - 1) ? q : 0;
        const unsigned p = (unsigned)(qc * nx + jcl);
        gv = ld_off(g, p);
        nv = ld_off(n2, p);
        if (odd) {
            const int I = (q + 1) >> 1;
            const bool Iok = I >= 1 && I < ncy;
            e0 = ld_off(ec, (unsigned)((Iok && cJ0 >= 0) ? I * ncx + cJ0 : 0));
            e1 = ld_off(ec, (unsigned)((Iok && cJ1 >= 0) ? I * ncx + cJ1 : 0));
        }
    };
#pragma unroll
    for (int s = 0; s < W; ++s) {
        gw[s] = uw[s] = wdw[s] = pew[s] = cplx<Tf>{};
        nw[s] = Tf(0);
        e0w[s] = e1w[s] = cplx<Tc>{};
    }
    static_for<P>([&](auto pc) {
        constexpr int s = decltype(pc)::value;
        load(q0 + s, gw[s], nw[s], e0w[s], e1w[s], (s & 1) == 0);
    });
#pragma unroll
    for (int t0 = 0; t0 < J0_STEPS; t0 += W) {
        static_for<W>([&](auto sc) {
            constexpr int s = decltype(sc)::value;
            constexpr int sm1 = (s + W - 1) % W, sm2 = (s + W - 2) % W, sp = (s + P) % W;
            // q0 is odd and W, t0 even: the parity of row q is that of s + 1
            constexpr bool odd = (s & 1) == 0;
            const int q = q0 + t0 + s;
            load(q + P, gw[sp], nw[sp], e0w[sp], e1w[sp], ((s + P) & 1) == 0);
            // P ec on row q: coarse rows q >> 1 (slot of the odd row before or of q itself
            // minus 2) and, for odd q, (q >> 1) + 1 (slot of q)
            cplx<Tc> pc;
            if constexpr (odd) {
                const cplx<Tc> a0 = e0w[sm2], a1 = e1w[sm2], b0 = e0w[s], b1 = e1w[s];
                pc = jodd ? Tc(0.25) * (((a0 + b0) + a1) + b1) : Tc(0.5) * (a0 + b0);
            } else {
                const cplx<Tc> a0 = e0w[sm1], a1 = e1w[sm1];
                pc = jodd ? Tc(0.5) * (a0 + a1) : a0;
            }
            // off the unknowns g and the coarse values were read as 0, so u = 0 there;
            // no branch, so that the loads ahead stay in flight
            const Tf ri = sponge_ramp<Tf>(q * G.s, G.nfy, Tf(G.inv_W));
            const cplx<Tf> wd = jac_wd<Tf>(G, nw[s], ri > rj ? ri : rj, w);
            pew[s] = ccast<Tf>(pc);
            wdw[s] = wd;
            uw[s] = wd * gw[s] + pew[s];
            // out on row q - 1
            const int r = q - 1;
            if (r >= rb && r <= re) {
                const cplx<Tf> c = uw[sm1];
                const cplx<Tf> nbs = ((uw[sm2] + uw[s]) + lane_prev(c)) + lane_next(c);
                const cplx<Tf> v = wdw[sm1] * (w2 * gw[sm1] + ih2 * nbs) + w1 * pew[sm1];
                if (own) out[(size_t)r * nx + j] = mk<Tf>(colok ? v.re : Tf(0), colok ? v.im : Tf(0));
            }
        });
    }
}

}  // namespace helm
