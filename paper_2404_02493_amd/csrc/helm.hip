// Host side of the Wave-ADR library: context and hierarchy setup, the cycle
// recursion (Algorithm 1), the ADR V-cycle with device-resident GMRES, the
// outer FGMRES / iterative refinement, and the C ABI of include/helm.h.
//
// The host only enqueues kernels; every grid operation runs in the kernels of
// kernels_*.hpp.  Scalars that steer the Krylov methods stay on the device,
// except that the outer solver reads one Hessenberg column per iteration.
#include <algorithm>
#include <array>
#include <cctype>
#include <atomic>
#include <complex>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <stdexcept>
#include <string>
#include <thread>
#include <vector>

#include "../../include/helm.h"
#include "kernels_tail.hpp"
#include "kernels_adjoint.hpp"
#include "kernels_wtail.hpp"
#include "kernels_eik.hpp"
#include "kernels_jac0.hpp"

namespace helm {

static thread_local std::string g_last_error;

struct Error : std::runtime_error {
    helm_status code;
    Error(helm_status c, const std::string& m) : std::runtime_error(m), code(c) {}
};

#define HIPCHK(expr)                                                                                      \
    do {                                                                                                  \
        hipError_t e_ = (expr);                                                                           \
        if (e_ != hipSuccess)                                                                             \
            throw Error(HELM_EHIP, std::string(#expr) + ": " + hipGetErrorString(e_) + " (line " +        \
                                       std::to_string(__LINE__) + ")");                                   \
    } while (0)

#define REQUIRE(cond, msg)                                   \
    do {                                                     \
        if (!(cond)) throw Error(HELM_EINVAL, (msg));        \
    } while (0)

struct WaveLevel {
    int nx = 0, ny = 0;    // nodes per row / per column
    Geom G{};
    bool f64 = false;      // this level computes in FP64
    void* n2 = nullptr;    // real, cycle precision (FP64 on f64 levels)
    void* g = nullptr;     // right-hand side (levels >= 2)
    void* u = nullptr;     // iterate (levels >= 2)
    void* ualt = nullptr;  // second iterate of the fused ADR steps (level 2)
    void* t = nullptr;     // Chebyshev scratch
    void* r = nullptr;
    void* d = nullptr;
    double lam = 0.0;      // spectral bound of A^*A
    double n2max = 0.0, n2mean = 0.0;
};

struct AdrLevel {
    int nx = 0, ny = 0;    // nodes per row / per column
    AdrGeom A{};
    void* px = nullptr;
    void* py = nullptr;
    void* c0 = nullptr;
    void* b = nullptr;
    void* balt = nullptr;  // second right-hand side of the fused ADR steps (level 2)
    void* x = nullptr;
    void* xalt = nullptr;  // second iterate for out-of-place s-step updates
    void* V[MAXM + 1] = {};
    KrylovScal* K = nullptr;
};

struct AdjState;

// A captured adjoint graph and the pointers and cycle count it was captured for.
struct AdjGraph {
    hipGraphExec_t exec = nullptr;
    const void* key[3] = {};
    int K = -1;
};
enum { ADJ_FULL = 0, ADJ_REC = 1, ADJ_REV = 2 };  // slots: record + reverse, record, reverse

// Chebyshev coefficient tables and per-level (lambda, alpha) in device memory (one copy per
// problem): la[0] = the Jacobi weight of level 1, la[2 l], la[2 l + 1] = (lambda_l, alpha_l);
// cheb[l][kind] rows of 3 doubles, row 0 = {1/theta, 0, 0},
// row s = {0, c1, c2} of step s; kind 0/1/2 = the pre, post and coarsest step counts.
constexpr int CHEB_ROWS = 65;
struct CycleDev {
    double la[2 * 16];
    double cheb[16][3][CHEB_ROWS * 3];
};

}  // namespace helm

struct helm_ctx_s {
    helm_desc d{};
    int L = 0;
    int LA = 0;  // coarsest level of the ADR V-cycle
    int LT = 0;  // first wave level run by the one-workgroup tail kernel (0 = none)
    bool f32 = false;  // cycle precision is complex64
    std::vector<void*> allocs;
    double* n2f = nullptr;  // fine n^2 (FP64)
    std::vector<helm::WaveLevel> wl;
    std::vector<helm::AdrLevel> al;
    void* car2 = nullptr;    // carrier e^{i sigma k phi} on level 2 (cycle precision)
    bool phase_set = false;
    bool phase_factored = false;  // ADR coefficients from the product rule (helm_eikonal)
    uint64_t data_gen = 0;  // counts changes of the phase and the weights (a recorded tape is
                            // reversible only while it is unchanged)
    // phase sets of the ADR correction: set 0 is the phase of helm_set_phase; helm_set_rays
    // fills nsets plane-wave sets and the m-th ADR step of a cycle uses set m mod nsets
    struct PhaseSet {
        void* px[16];
        void* py[16];
        void* c0[16];
        void* car;
    };
    std::vector<PhaseSet> sets;
    int nsets = 1;
    std::vector<double> w, w_default;
    void* ws1 = nullptr;     // second level-1 iterate (cycle precision)
    double* partials = nullptr;
    size_t partials_cap = 0;  // doubles
    double* dscal = nullptr;  // small device scratch (norms)
    helm::CycleDev* cdev = nullptr;  // Chebyshev tables and level (lambda, alpha) on the device
    helm::BatchIdx bi{};             // problems served by each launch (zero: this context alone)
    // batch arena: the context's device buffers are carved from [arena, arena + arena_cap)
    // in allocation order (its region of a batch class); count_bytes sums every allocation
    char* arena = nullptr;
    size_t arena_cap = 0, arena_used = 0, count_bytes = 0;
    void* bg = nullptr;  // batch staging of g and u (complex128, fine grid)
    void* bu = nullptr;
    helm::KrylovScal* Kout = nullptr;
    helm::KrylovScal* Kin = nullptr;
    // outer FGMRES (complex128) and inner (cycle precision, iterative refinement)
    void* fV[helm::MAXM + 1] = {};
    void* fZ[helm::MAXM] = {};
    void* iV[helm::MAXM + 1] = {};
    void* iZ[helm::MAXM] = {};
    void* cyc_g = nullptr;   // cycle-precision staging (mode 0 with complex64 cycles)
    void* cyc_u = nullptr;
    void* rbuf = nullptr;    // FP64 residual (mode 1)
    double* hcol = nullptr;  // pinned host copies of the outer Hessenberg columns
    hipEvent_t col_ev[helm::MAXM] = {};
    void* dbuf = nullptr;    // inner correction (mode 1)
    helm::AdjState* adj = nullptr;  // adjoint tape (allocated on first use)
    // the adjoint's captured work: ADJ_FULL all K cycles with one tape each (K) or the
    // recording and reverse of one cycle (K = 0); ADJ_REC the recording of K cycles;
    // ADJ_REV their reverse; each keyed by (g, checkpoints) and K
    helm::AdjGraph adj_graph[3];
    // launch shapes chosen by the autotuner (0 = built-in default)
    struct Tuning {
        int sstep_rows[16] = {};    // s-step form on ADR level l: steps per marching unit, 1/2 tiles, 0 default
        int fgmres_blocks = 0;      // blocks of the outer FGMRES passes on the fine grid
    } tn;
    // captured cycles, keyed by the (g, u_in, u_out) pointers they were captured with
    struct GraphEntry {
        const void* g;
        const void* uin;
        void* uout;
        hipGraphExec_t exec;
    };
    std::vector<GraphEntry> graphs;
    hipStream_t cap_stream = nullptr;  // library-owned stream used only for capture
    // per-launch timing with HIP events and the algorithmic bytes of each launch
    struct Prof {
        struct Rec {
            const char* name;
            int grid;
            double bytes;
            hipEvent_t e0, e1;
        };
        bool on = false;
        std::vector<Rec> recs;
        std::vector<hipEvent_t> pool;
        size_t used = 0;
        hipEvent_t next(hipStream_t st) {
            if (used == pool.size()) {
                // timing-only events: no system-scope fence, so recording one does not
                // write back and invalidate the caches between the timed launches
                hipEvent_t e;
                if (hipEventCreateWithFlags(&e, hipEventDisableSystemFence) != hipSuccess) return nullptr;
                pool.push_back(e);
            }
            hipEvent_t e = pool[used++];
            (void)hipEventRecord(e, st);
            return e;
        }
    } prof;
};

// A batch of independent problems (see batch.hpp): one context per problem and
// one stream + host thread per lane.
struct helm_batch_s {
    // problems of equal descriptors, built region by region in one arena, solved in lockstep
    struct Class {
        std::vector<int> probs;     // problem indices, region q holds probs[q]
        char* arena = nullptr;
        size_t stride = 0;          // bytes per region
        double* dg = nullptr;       // device gather buffer (per-problem scalars and columns)
        double* hg = nullptr;       // pinned host copy of it
        hipEvent_t ev[helm::MAXM + 1] = {};
    };
    std::vector<Class> classes;
    std::vector<int> last_class;  // per problem: the class it ran in at the last solve, -1 alone
    std::vector<helm_ctx> ctx;
    int lanes = 0;
    int device = 0;
    std::vector<hipStream_t> streams;
    std::vector<hipEvent_t> events;  // one per lane
    hipEvent_t ev_in = nullptr;
};

// Launch with optional per-launch event timing (name = kernel expression).  LAUNCH
// appends the context's batch index (the problems the launch serves, gridDim.z of them;
// one for a single problem) to the kernel arguments; LAUNCH_NB is for kernels that
// serve one problem only.
#define LAUNCH_IMPL(CTX, BYTES, KERN, GRID, BLK, ST, ...)                               \
    do {                                                                                \
        hipEvent_t e0_ = nullptr;                                                       \
        if ((CTX)->prof.on) e0_ = (CTX)->prof.next(ST);                                 \
        hipLaunchKernelGGL(KERN, GRID, BLK, 0, ST, __VA_ARGS__);                        \
        if ((CTX)->prof.on && e0_) {                                                    \
            hipEvent_t e1_ = (CTX)->prof.next(ST);                                      \
            (CTX)->prof.recs.push_back({#KERN, (int)dim3(GRID).x, (double)(BYTES), e0_, e1_}); \
        }                                                                               \
    } while (0)
#define LAUNCH(CTX, BYTES, KERN, GRID, BLK, ST, ...)                                                       \
    LAUNCH_IMPL(CTX, BYTES, KERN, helm::bgrid(CTX, GRID), BLK, ST, __VA_ARGS__, (CTX)->bi)
#define LAUNCH_NB(CTX, BYTES, KERN, GRID, BLK, ST, ...) LAUNCH_IMPL(CTX, BYTES, KERN, GRID, BLK, ST, __VA_ARGS__)

namespace helm {

// Grid of a launch: gridDim.z = the number of problems the context's batch index serves.
static inline dim3 bgrid(const helm_ctx c, dim3 g) {
    g.z = c->bi.n > 1 ? (unsigned)c->bi.n : 1u;
    return g;
}

static void* dalloc(helm_ctx c, size_t bytes) {
    void* p = nullptr;
    if (bytes == 0) bytes = 256;
    const size_t rb = (bytes + 255) & ~size_t(255);
    c->count_bytes += rb;
    if (c->arena && c->arena_used + rb <= c->arena_cap) {
        p = c->arena + c->arena_used;
        c->arena_used += rb;
        return p;
    }
    hipError_t e = hipMalloc(&p, bytes);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        throw Error(HELM_ENOMEM, "hipMalloc of " + std::to_string(bytes) + " bytes failed: " + hipGetErrorString(e));
    }
    c->allocs.push_back(p);
    return p;
}

static inline dim3 tile_block() { return dim3(TX, TWY, 1); }
static inline int flat_blocks(size_t N, int cap = 2048) {
    size_t b = (N + BLOCK - 1) / BLOCK;
    return (int)std::max<size_t>(1, std::min<size_t>(b, (size_t)cap));
}

// Nodes per row / per column of level l (the fine grid has d.n x d.ny; setup stores
// d.ny = d.n for a square grid).
static inline int lnx(const helm_ctx c, int level) { return c->d.n >> (level - 1); }
static inline int lny(const helm_ctx c, int level) { return c->d.ny >> (level - 1); }
// 1/h of level l: h = 2^(l-1) / max(n, ny)
static inline double inv_h(const helm_ctx c, int level) { return double(std::max(lnx(c, level), lny(c, level))); }

static Geom make_geom(const helm_ctx c, int level) {
    Geom G{};
    G.nx = lnx(c, level);
    G.ny = lny(c, level);
    G.s = 1 << (level - 1);
    G.nfx = c->d.n;
    G.nfy = c->d.ny;
    G.W = c->d.damping_cells;
    G.inv_W = 1.0 / double(G.W);
    G.inv_h2 = inv_h(c, level) * inv_h(c, level);
    G.k2 = c->d.k * c->d.k;
    G.sig_str = double(c->d.sign) * c->d.damping_strength;
    G.sig_shift = double(c->d.sign) * (c->d.shift + c->d.cycle_shift);
    return G;
}

// Level-1 geometry of the system operator (without the cycle-only shift): the outer
// Krylov solver, the FP64 residual and the loss.
static Geom make_geom_sys(const helm_ctx c) {
    Geom G = make_geom(c, 1);
    G.sig_shift = double(c->d.sign) * c->d.shift;
    return G;
}

static AdrGeom make_adr_geom(const helm_ctx c, int level) {
    AdrGeom A{};
    A.nx = lnx(c, level);
    A.ny = lny(c, level);
    A.inv_h2 = inv_h(c, level) * inv_h(c, level);
    A.inv_2h = 0.5 * inv_h(c, level);
    A.two_sk = 2.0 * double(c->d.sign) * c->d.k;
    return A;
}

static inline double NN2(int nx, int ny) { return double(nx) * double(ny); }

static size_t csize(bool f64) { return f64 ? sizeof(c128) : sizeof(c64); }
static size_t rsize(bool f64) { return f64 ? sizeof(double) : sizeof(float); }

static int nv_bucket(int m) { return m <= 4 ? 4 : (m <= 12 ? 12 : MAXM); }

// ------------------------------------------------------------------ default weights
// The sine modes of a level with nx x ny nodes and spacing h have the symbol
// (4/h^2)(sin^2(pi a/(2 nx)) + sin^2(pi b/(2 ny))) - k^2 n2mean.
static double median_alpha(double k, double n2mean, int nx, int ny, double h, double lam) {
    auto sines = [](int m) {
        std::vector<double> s(m - 1);
        for (int a = 1; a < m; ++a) {
            double v = std::sin(a * M_PI / (2.0 * m));
            s[a - 1] = v * v;
        }
        return s;
    };
    const std::vector<double> sx = sines(nx), sy = sines(ny);
    std::vector<double> vals(sx.size() * sy.size());
    const double c4 = 4.0 / (h * h), kk = k * k * n2mean;
    size_t q = 0;
    for (size_t b = 0; b < sy.size(); ++b)
        for (size_t a = 0; a < sx.size(); ++a) {
            double sig = c4 * (sy[b] + sx[a]) - kk;
            vals[q++] = sig * sig;
        }
    size_t mid = (vals.size() - 1) / 2;
    std::nth_element(vals.begin(), vals.begin() + mid, vals.end());
    double med = vals[mid];
    if (vals.size() % 2 == 0) {
        double hi = *std::min_element(vals.begin() + mid + 1, vals.end());
        med = 0.5 * (med + hi);
    }
    return std::max(1.0, lam / med);
}

// f(std::integral_constant<int, J>{}) for the runtime value j = J in [0, N).
template <int N, int J = 0, typename F>
static void static_for_host(int j, F&& f) {
    if constexpr (J < N) {
        if (j == J)
            f(std::integral_constant<int, J>{});
        else
            static_for_host<N, J + 1>(j, f);
    }
}

// ------------------------------------------------------------------ Krylov finalize helper
template <int NV>
static void krylov_fin(helm_ctx c, hipStream_t st, int nblk, int op, int jj, int m, KrylovScal* K, double tol) {
    if (op == FIN_INIT || op == FIN_ORTH2) {
        LAUNCH(c, 8.0 * nblk, (k_krylov_finalize<2>), dim3(1), dim3(FBLOCK), st, (const double*)c->partials, nblk, op,
               jj, m, K, tol);
    } else {
        LAUNCH(c, 16.0 * nblk * (jj + 1), (k_krylov_finalize<2 * NV + 2>), dim3(1), dim3(FBLOCK), st,
               (const double*)c->partials, nblk, op, jj, m, K, tol);
    }
}

static void use_set(helm_ctx c, int m);

// ------------------------------------------------------------------ engine
template <typename T>
struct Engine {
    helm_ctx c;
    hipStream_t st;
    using C = cplx<T>;

    Engine(helm_ctx ctx, hipStream_t s) : c(ctx), st(s) {}

    size_t N(int level) const { return (size_t)lnx(c, level) * (size_t)lny(c, level); }

    // ---- generic launches on a level of precision P
    template <typename P>
    void residual(const Geom& G, const void* n2, const void* g, const void* u, void* r) {
        LAUNCH(c, ((u ? 3 : 2) * sizeof(cplx<P>) + (u ? sizeof(P) : 0)) * NN2(G.nx, G.ny), (k_residual<P>), dim3(tiles_of(G.nx, G.ny)), tile_block(), st, G, (const P*)n2,
                           (const cplx<P>*)g, (const cplx<P>*)u, (cplx<P>*)r);
    }
    template <typename P>
    void applyA(const Geom& G, const void* n2, const void* x, void* y, int conj_k) {
        LAUNCH(c, (2 * sizeof(cplx<P>) + sizeof(P)) * NN2(G.nx, G.ny), (k_apply_A<P>), dim3(tiles_of(G.nx, G.ny)), tile_block(), st, G, (const P*)n2,
                           (const cplx<P>*)x, (cplx<P>*)y, conj_k);
    }
    template <typename P>
    void zero(void* y, size_t n) {
        LAUNCH(c, sizeof(cplx<P>) * double(n), (k_zero<P>), dim3(flat_blocks(n)), dim3(BLOCK), st, n, (cplx<P>*)y);
    }

    // Coefficient table of level l for m steps (see CycleDev; the pre, post and coarsest
    // counts of the descriptor).
    const double* cheb_table(int l, int m, double alpha) const {
        const int kind = m == c->d.cheb_pre ? 0 : m == c->d.cheb_post ? 1 : m == c->d.cheb_coarse ? 2 : -1;
        REQUIRE(kind >= 0, "Chebyshev step count without a coefficient table");
        REQUIRE(alpha == c->w[l - 1], "Chebyshev alpha other than the level's weight");
        return c->cdev->cheb[l][kind];
    }

    template <typename P>
    void chebyshev(int l, const void* g, void* u, bool u_zero, double alpha, int m) {
        WaveLevel& W = c->wl[l];
        const Geom& G = W.G;
        const size_t n = N(l);
        const double* tab = cheb_table(l, m, alpha);
        // with two steps or more the first fused step takes u = 0 itself and the last one
        // adds the final d (no zero fill, no closing axpy)
        const bool fused_ends = m >= 2;
        if (u_zero && !fused_ends) zero<P>(u, n);
        if (u_zero)
            LAUNCH(c, (3 * sizeof(cplx<P>) + sizeof(P)) * NN2(G.nx, G.ny), (k_cheb_start<P>), dim3(tiles_of(G.nx, G.ny)),
                   tile_block(), st, G, (const P*)W.n2, (const cplx<P>*)g, (cplx<P>*)W.r, (cplx<P>*)W.d, tab);
        else
            LAUNCH(c, (4 * sizeof(cplx<P>) + sizeof(P)) * NN2(G.nx, G.ny), (k_cheb_start_res<P>), dim3(tiles_of(G.nx, G.ny)),
                   tile_block(), st, G, (const P*)W.n2, (const cplx<P>*)g, (const cplx<P>*)u, (cplx<P>*)W.r,
                   (cplx<P>*)W.d, tab);
        void* dcur = W.d;  // d alternates between W.d and W.t
        void* dnext = W.t;
        for (int step = 1; step <= m; ++step) {
            if (step < m) {
                const int mode = (step == 1 && u_zero ? CHEB_UZERO : 0) | (step == m - 1 ? CHEB_LAST : 0);
                const int nb = 6 - ((mode & CHEB_UZERO) ? 1 : 0) - ((mode & CHEB_LAST) ? 2 : 0);
                LAUNCH(c, (nb * sizeof(cplx<P>) + sizeof(P)) * NN2(G.nx, G.ny), (k_cheb_fused<P>), dim3(tiles_of(G.nx, G.ny)),
                       tile_block(), st, G, (const P*)W.n2, (const cplx<P>*)dcur, (cplx<P>*)dnext, (cplx<P>*)W.r,
                       (cplx<P>*)u, tab + 3 * step, mode);
                std::swap(dcur, dnext);
            } else if (!fused_ends) {
                LAUNCH(c, 3 * sizeof(cplx<P>) * double(n), (k_axpy<P>), dim3(flat_blocks(n)), dim3(BLOCK), st, n, P(1),
                                   (const cplx<P>*)dcur, (cplx<P>*)u);
            }
        }
    }

    // rc = R (g - A u) from level l (precision Pf) to level l+1 (precision Pc)
    template <typename Pf, typename Pc>
    void resid_restrict(int l, const void* g, const void* u, void* rc) {
        const Geom& G = c->wl[l].G;
        LAUNCH(c, (u ? 2 * sizeof(cplx<Pf>) + sizeof(Pf) : sizeof(cplx<Pf>)) * NN2(G.nx, G.ny) + sizeof(cplx<Pc>) * NN2(G.nx / 2, G.ny / 2), (k_resid_restrict<Pf, Pc>), dim3(rr_blocks(G.nx, G.ny)), dim3(BLOCK), st, G,
                           (const Pf*)c->wl[l].n2, (const cplx<Pf>*)g, (const cplx<Pf>*)u, (cplx<Pc>*)rc);
    }
    template <typename Pc, typename Pf>
    void prolong_add(int l, const void* ec, void* u, bool assign = false) {
        const int nx = c->wl[l].nx, ny = c->wl[l].ny;
        const size_t np = (size_t)ny * (nx / 2);
        LAUNCH(c, (assign ? 1 : 2) * sizeof(cplx<Pf>) * NN2(nx, ny) + sizeof(cplx<Pc>) * NN2(nx / 2, ny / 2),
               (k_prolong_pairs<Pc, Pf>), dim3(flat_blocks(np)), dim3(BLOCK), st, nx, ny, (const cplx<Pc>*)ec,
               (cplx<Pf>*)u, assign ? 1 : 0);
    }

    void restrict_down(int l, const void* g, const void* u, void* rc) {
        if (c->wl[l + 1].f64)
            resid_restrict<T, double>(l, g, u, rc);
        else
            resid_restrict<T, T>(l, g, u, rc);
    }
    void prolong_up(int l, const void* ec, void* u, bool assign = false) {
        if (c->wl[l + 1].f64)
            prolong_add<double, T>(l, ec, u, assign);
        else
            prolong_add<T, T>(l, ec, u, assign);
    }

    // ---- the coarsest wave level (always FP64)
    void coarsest(int l) {
        WaveLevel& W = c->wl[l];
        chebyshev<double>(l, W.g, W.u, true, c->w[l - 1], c->d.cheb_coarse);
    }

    // ---- levels LT..L in one workgroup (u_LT from g_LT, zero initial iterate)
    void wave_tail(int l0) {
        TailWaveArgs a{};
        for (int l = l0; l <= c->L; ++l) {
            WaveLevel& W = c->wl[l];
            TailWaveLevel& t = a.lv[l];
            t.G = W.G;
            t.f64 = W.f64 ? 1 : 0;
            t.n2 = W.n2;
            t.g = W.g;
            t.u = W.u;
            t.r = W.r;
            t.d = W.d;
            t.t = W.t;
            t.la = c->cdev->la + 2 * l;
        }
        a.l0 = l0;
        a.L = c->L;
        a.cheb_pre = c->d.cheb_pre;
        a.cheb_post = c->d.cheb_post;
        a.cheb_coarse = c->d.cheb_coarse;
        a.level3_literal = c->d.level3_literal;
        double bytes = 0.0;
        for (int l = l0; l <= c->L; ++l) bytes += 8.0 * csize(c->wl[l].f64) * NN2(c->wl[l].nx, c->wl[l].ny);
        LAUNCH(c, bytes, (k_wave_tail<T>), dim3(1), dim3(WT_THREADS), st, a);
    }

    // ---- one cycle on level l >= 2 with zero initial iterate: u_l from g_l
    void cycle_coarse(int l) {
        WaveLevel& W = c->wl[l];
        const int L = c->L;
        if (c->LT > 0 && l >= c->LT) {
            wave_tail(l);
            return;
        }
        if (l == L) {
            coarsest(l);
            return;
        }
        bool u_zero = true;
        if (l == 3) {
            // no pre-smoothing on level 3
        } else {
            chebyshev<T>(l, W.g, W.u, true, c->w[l - 1], c->d.cheb_pre);
            u_zero = false;
        }
        restrict_down(l, W.g, u_zero ? nullptr : W.u, c->wl[l + 1].g);
        cycle_coarse(l + 1);
        prolong_up(l, c->wl[l + 1].u, W.u, u_zero);  // u = P e when no pre-smoothing ran
        if (l == 2) {
            chebyshev<T>(l, W.g, W.u, false, c->w[1], c->d.cheb_post);
            if (c->d.adr_steps > 0 && L >= 3) adr_steps(c->d.adr_steps);
        } else if (l == 3 && !c->d.level3_literal) {
            // no post-smoothing on level 3
        } else {
            chebyshev<T>(l, W.g, W.u, false, c->w[l - 1], c->d.cheb_post);
        }
    }

    // ---- fine-grid cycle: u_out = C(u_in, g); u_in may be null (zero)
    void cycle(const void* g, const void* u_in, void* u_out) {
        WaveLevel& W = c->wl[1];
        const Geom& G = W.G;
        const double* w0 = c->cdev->la;  // la[0]: the Jacobi weight of this problem
        if (u_in == nullptr) {
            // the zero-start Jacobi sweep is recomputed inside the restriction and the
            // post-smoother instead of being stored
            const bool c64 = c->wl[2].f64;
            const double bc = c64 ? 16.0 : sizeof(C);
            if (c64)
                LAUNCH(c, (sizeof(C) + sizeof(T)) * NN2(G.nx, G.ny) + bc * NN2(G.nx / 2, G.ny / 2), (k_jac0_restrict<T, double>),
                       dim3(jac0r_units(G.nx, G.ny)), dim3(64), st, G, (const T*)W.n2, (const C*)g, w0,
                       (c128*)c->wl[2].g);
            else
                LAUNCH(c, (sizeof(C) + sizeof(T)) * NN2(G.nx, G.ny) + bc * NN2(G.nx / 2, G.ny / 2), (k_jac0_restrict<T, T>),
                       dim3(jac0r_units(G.nx, G.ny)), dim3(64), st, G, (const T*)W.n2, (const C*)g, w0, (C*)c->wl[2].g);
            cycle_coarse(2);
            if (c64)
                LAUNCH(c, (2 * sizeof(C) + sizeof(T)) * NN2(G.nx, G.ny) + bc * NN2(G.nx / 2, G.ny / 2), (k_jac0_prolong_jacobi<double, T>),
                       dim3(jac0p_units(G.nx, G.ny)), dim3(64), st, G, (const T*)W.n2, (const C*)g,
                       (const c128*)c->wl[2].u, w0, (C*)u_out);
            else
                LAUNCH(c, (2 * sizeof(C) + sizeof(T)) * NN2(G.nx, G.ny) + bc * NN2(G.nx / 2, G.ny / 2), (k_jac0_prolong_jacobi<T, T>),
                       dim3(jac0p_units(G.nx, G.ny)), dim3(64), st, G, (const T*)W.n2, (const C*)g,
                       (const C*)c->wl[2].u, w0, (C*)u_out);
            return;
        }
        LAUNCH(c, ((u_in ? 3 : 2) * sizeof(C) + sizeof(T)) * NN2(G.nx, G.ny), (k_jacobi<T>), dim3(tiles_of(G.nx, G.ny)), tile_block(), st, G, (const T*)W.n2,
                           (const C*)g, (const C*)u_in, (C*)c->ws1, w0);
        restrict_down(1, g, c->ws1, c->wl[2].g);
        cycle_coarse(2);
        prolong_up(1, c->wl[2].u, c->ws1);
        LAUNCH(c, (3 * sizeof(C) + sizeof(T)) * NN2(G.nx, G.ny), (k_jacobi<T>), dim3(tiles_of(G.nx, G.ny)), tile_block(), st, G, (const T*)W.n2,
                           (const C*)g, (const C*)c->ws1, (C*)u_out, w0);
    }

    // ---- ADR corrections on level 2 (M = adr_steps of them)
    // Each step: r = g - A u, demodulate, one ADR V-cycle, u += a e^{i theta}.  When the
    // post-smoother of level 2 runs in s-step form, its second pass also re-modulates
    // and adds the correction and demodulates the next step's right-hand side (the
    // last step only adds), writing the other buffer of u and b; the pointers end on
    // the buffers they started on.
    bool adr_fused() const {
        const int m = c->d.gmres_m;
        return c->LA > 2 && m <= 3 && !c->d.gmres_arnoldi && c->wl[2].ualt && c->al[2].balt && c->nsets == 1;
    }
    ModArgs<T> mod_args(void* uout, void* bout) {
        WaveLevel& W = c->wl[2];
        ModArgs<T> a{};
        a.G = W.G;
        a.car = (const C*)c->car2;
        a.n2 = (const T*)W.n2;
        a.g = (const C*)W.g;
        a.u = (const C*)W.u;
        a.uout = (C*)uout;
        a.bout = (C*)bout;
        return a;
    }
    void adr_steps(int M) {
        WaveLevel& W = c->wl[2];
        AdrLevel& A = c->al[2];
        void* const u_home = W.u;
        void* const b_home = A.b;
        const bool fused = adr_fused();
        for (int s = 0; s < M; ++s) {
            if (c->nsets > 1) use_set(c, s % c->nsets);
            if (s == 0 || !fused)
                LAUNCH(c, (4 * sizeof(C) + sizeof(T)) * NN2(W.nx, W.ny), (k_adr_demod<T>), dim3(tiles_of(W.nx, W.ny)), tile_block(),
                       st, W.G, (const T*)W.n2, (const C*)W.g, (const C*)W.u, (const C*)c->car2, (C*)A.b);
            if (!fused) {
                adr_vcycle(2);
                LAUNCH(c, 4 * sizeof(C) * double(N(2)), (k_adr_modadd<T>), dim3(flat_blocks(N(2))),
                       dim3(BLOCK), st, N(2), (const C*)A.x, (const C*)c->car2, (C*)W.u);
                continue;
            }
            if (s + 1 < M) {
                const ModArgs<T> ma = mod_args(W.u == u_home ? W.ualt : u_home, A.b == b_home ? A.balt : b_home);
                adr_vcycle(2, EPI_MODRD, &ma);
                std::swap(W.u, W.ualt);
                std::swap(A.b, A.balt);
            } else {
                const ModArgs<T> ma = mod_args(u_home, nullptr);
                adr_vcycle(2, EPI_MOD, &ma);
                if (W.u != u_home) std::swap(W.u, W.ualt);
            }
        }
        if (A.b != b_home) std::swap(A.b, A.balt);
        if (c->nsets > 1) use_set(c, 0);
    }

    // GMRES on a small level in one workgroup (the coarsest ADR level), if it fits.
    // the coarsest level's GMRES runs in one workgroup (gmres_block)
    bool block_form(int l, int m) const {
        const AdrLevel& A = c->al[l];
        return l == c->LA && std::max(A.nx, A.ny) <= c->d.tail_n && (size_t)A.nx * A.ny <= 4 * 1024 && m <= 12;
    }
    bool gmres_block(int l, int m, bool x0_zero) {
        AdrLevel& A = c->al[l];
        if (!block_form(l, m)) return false;
        BlockLevel<T> t{};
        t.A = A.A;
        t.px = (const T*)A.px;
        t.py = (const T*)A.py;
        t.c0 = (const C*)A.c0;
        t.b = (const C*)A.b;
        t.x = (C*)A.x;
        t.V = (C*)A.V[0];
        t.m = m;
        const double bytes = (3.0 * m + 4.0) * sizeof(C) * NN2(A.nx, A.ny);
        if (m <= 4)
            LAUNCH(c, bytes, (k_gmres_block<T, 1024, 4, 4096>), dim3(1), dim3(1024), st, t, x0_zero ? 1 : 0, 1e-14);
        else
            LAUNCH(c, bytes, (k_gmres_block<T, 512, 12, 4096>), dim3(1), dim3(512), st, t, x0_zero ? 1 : 0, 1e-14);
        return true;
    }

    // One ADR V-cycle from x = 0 on levels l..LA (result in A.x, or handed to the
    // epilogue epi of the last smoother of level l).
    // ADR V-cycle from level l (result in A.x); with pinto, P x_l is added into pinto (the
    // iterate of level l - 1), by the smoother's last pass itself in the tile form (x_l is
    // then not stored).
    void adr_vcycle(int l, int epi = EPI_X, const ModArgs<T>* ma = nullptr, void* pinto = nullptr) {
        AdrLevel& A = c->al[l];
        const bool coarse = l == c->LA;
        const int m = coarse ? c->d.gmres_coarse_m : c->d.gmres_m;
        if (!coarse) {
            presmooth_restrict(l);
            adr_vcycle(l + 1, EPI_X, nullptr, A.x);
        }
        if (pinto && epi == EPI_X && sstep_form(m) && sstep_tile_edge(l) && !(coarse && block_form(l, m))) {
            switch (m) {
                case 1: smooth_prolong_tile<1>(l, coarse, pinto); break;
                case 2: smooth_prolong_tile<2>(l, coarse, pinto); break;
                case 3: smooth_prolong_tile<3>(l, coarse, pinto); break;
                default: smooth_prolong_tile<4>(l, coarse, pinto); break;
            }
            return;
        }
        if (coarse)
            gmres(l, m, true);
        else
            gmres(l, m, false, epi, ma);
        if (pinto) {
            const int fx = c->al[l - 1].nx, fy = c->al[l - 1].ny;
            LAUNCH(c, 2 * sizeof(C) * NN2(fx, fy) + sizeof(C) * NN2(fx / 2, fy / 2), (k_prolong_add<T, T>),
                   dim3(tiles_of(fx, fy)), tile_block(), st, fx, fy, (const C*)A.x, (C*)pinto);
        }
    }
    template <int MM>
    void smooth_prolong_tile(int l, bool x0_zero, void* pinto) {
        AdrLevel& A = c->al[l];
        const int S = sstep_steps(l), tt = sstep_tile_edge(l);
        const double bytes = ((x0_zero ? 2 : 3) * sizeof(C) + 2 * sizeof(T)) * NN2(A.nx, A.ny) + 2 * sizeof(C) * NN2(2 * A.nx, 2 * A.ny);
        if (x0_zero)
            sstep_gram_solve<MM, false>(l, S, tt);
        else
            sstep_gram_solve<MM, true>(l, S, tt);
        with_edge(tt, [&](auto e) {
            constexpr int TT = decltype(e)::value;
            if (x0_zero)
                LAUNCH(c, bytes, (k_sstep_combine_tile_pa<T, MM, false, TT>),
                       dim3(Tile<MM, false, false, TT, 1>::tiles(A.nx, A.ny)), dim3(BLOCK), st, A.A, (const T*)A.px,
                       (const T*)A.py, (const C*)A.c0, (const C*)A.b, (const C*)nullptr, (const KrylovScal*)A.K,
                       (C*)pinto);
            else
                LAUNCH(c, bytes, (k_sstep_combine_tile_pa<T, MM, true, TT>),
                       dim3(Tile<MM, true, false, TT, 1>::tiles(A.nx, A.ny)), dim3(BLOCK), st, A.A, (const T*)A.px,
                       (const T*)A.py, (const C*)A.c0, (const C*)A.b, (const C*)A.x, (const KrylovScal*)A.K,
                       (C*)pinto);
        });
    }

    // Pre-smoother from zero on level l < LA and b_{l+1} = R(b - M x): in the marching
    // s-step form the second pass also forms and restricts the residual.
    void presmooth_restrict(int l) {
        AdrLevel& A = c->al[l];
        const int m = c->d.gmres_m;
        if (sstep_form(m)) {
            switch (m) {
                case 1: presmooth_restrict_sstep<1>(l); break;
                case 2: presmooth_restrict_sstep<2>(l); break;
                case 3: presmooth_restrict_sstep<3>(l); break;
                default: presmooth_restrict_sstep<4>(l); break;
            }
            return;
        }
        gmres(l, m, true);
        LAUNCH(c, (3 * sizeof(C) + 2 * sizeof(T)) * NN2(A.nx, A.ny) + sizeof(C) * NN2(A.nx / 2, A.ny / 2), (k_adr_resid_restrict<T>),
               dim3(rr_blocks(A.nx, A.ny)), dim3(BLOCK), st, A.A, (const T*)A.px, (const T*)A.py, (const C*)A.c0,
               (const C*)A.b, (const C*)A.x, (C*)c->al[l + 1].b);
    }
    template <int MM>
    void presmooth_restrict_sstep(int l) {
        AdrLevel& A = c->al[l];
        const int S = sstep_steps(l), tt = sstep_tile_edge(l);
        const double bytes = (3 * sizeof(C) + 2 * sizeof(T)) * NN2(A.nx, A.ny) + sizeof(C) * NN2(A.nx / 2, A.ny / 2);
        sstep_gram_solve<MM, false>(l, S, tt);
        if (tt) {
            with_edge(tt, [&](auto e) {
                constexpr int TT = decltype(e)::value;
                LAUNCH(c, bytes, (k_sstep_combine_tile_rr<T, MM, TT>), dim3(Tile<MM, false, true, TT, 1>::tiles(A.nx, A.ny)),
                       dim3(BLOCK), st, A.A, (const T*)A.px, (const T*)A.py, (const C*)A.c0, (const C*)A.b,
                       (const KrylovScal*)A.K, (C*)A.x, (C*)c->al[l + 1].b);
            });
        } else {
            LAUNCH(c, bytes, (k_sstep_combine_rr<T, MM>), dim3(March<MM, false, true, 1>::units(A.nx, A.ny, S)), dim3(64),
                   st, A.A, S, (const T*)A.px, (const T*)A.py, (const C*)A.c0, (const C*)A.b,
                   (const KrylovScal*)A.K, (C*)A.x, (C*)c->al[l + 1].b);
        }
    }

    template <int NV>
    void gmres_nv(int l, int m, bool x0_zero) {
        AdrLevel& A = c->al[l];
        const size_t n = N(l);
        VecSet<T> V{};
        V.v[0] = (const C*)(x0_zero ? A.b : A.V[0]);
        for (int i = 1; i <= m; ++i) V.v[i] = (const C*)A.V[i];
        const int nbf = flat_blocks(n, MAXRED), nbt = red_blocks(A.nx, A.ny);
        if (x0_zero) {
            LAUNCH(c, sizeof(C) * double(n), (k_krylov_init_norm<T>), dim3(nbf), dim3(BLOCK), st, n, (const C*)A.b,
                   c->partials);
            krylov_fin<NV>(c, st, nbf, FIN_INIT, 0, m, A.K, 0.0);
        } else {
            LAUNCH(c, (4 * sizeof(C) + 2 * sizeof(T)) * NN2(A.nx, A.ny), (k_adr_residual_init<T>), dim3(nbt), tile_block(), st,
                   A.A, (const T*)A.px, (const T*)A.py, (const C*)A.c0, (const C*)A.b, (const C*)A.x, (C*)A.V[0],
                   c->partials);
            krylov_fin<NV>(c, st, nbt, FIN_INIT, 0, m, A.K, 0.0);
        }
        for (int j = 0; j < m; ++j) {
            LAUNCH(c, ((j + 3) * sizeof(C) + 2 * sizeof(T)) * NN2(A.nx, A.ny), (k_arnoldi_adr<T, NV>), dim3(nbt), tile_block(),
                   st, A.A, (const T*)A.px, (const T*)A.py, (const C*)A.c0, V, j, (C*)A.V[j + 1],
                   (const KrylovScal*)A.K, c->partials);
            krylov_fin<NV>(c, st, nbt, FIN_MV, j, m, A.K, 0.0);
            LAUNCH(c, (j + 3) * sizeof(C) * double(n), (k_orth_pass1<T, NV>), dim3(nbf), dim3(BLOCK), st, n, V, j,
                   (C*)A.V[j + 1], (const KrylovScal*)A.K, c->partials);
            krylov_fin<NV>(c, st, nbf, FIN_ORTH1, j, m, A.K, 0.0);
            LAUNCH(c, (j + 3) * sizeof(C) * double(n), (k_orth_pass2<T, NV>), dim3(nbf), dim3(BLOCK), st, n, V, j,
                   (C*)A.V[j + 1], (const KrylovScal*)A.K, c->partials);
            krylov_fin<NV>(c, st, nbf, FIN_ORTH2, j, m, A.K, 1e-14);
        }
        LAUNCH(c, (m + 1 + (x0_zero ? 0 : 1)) * sizeof(C) * double(n), (k_krylov_combine<T, NV>), dim3(flat_blocks(n)), dim3(BLOCK), st, n, V,
                           (const KrylovScal*)A.K, (const C*)(x0_zero ? nullptr : A.x), (C*)A.x, 0);
    }
    // Steps per unit of the marching s-step passes on ADR level l (a multiple of 8; a
    // unit covers that many rows minus twice its halo): the tuned value, else the
    // shortest (24..128) that keeps the Gram pass at 2048 wavefronts or fewer.
    int sstep_steps(int l) const {
        if (c->tn.sstep_rows[l] >= 16) return c->tn.sstep_rows[l];
        const int nx = c->al[l].nx, ny = c->al[l].ny;
        int S = 24;
        while (S < 128 && March<3, true, true>::units(nx, ny, S) > 2048) S += 8;
        return S;
    }
    // Tile edge of the overlapped-tile form on level l (tuned value 1: 16, 2: 32), 0 when
    // the level marches.
    // Untuned default (measured on 4096^2): march from 2048^2 nodes up, 32 x 32 tiles from
    // 1024^2, 16 x 16 tiles below.
    int sstep_tile_edge(int l) const {
        const int v = c->tn.sstep_rows[l];
        if (v == 0) {
            const size_t a = (size_t)c->al[l].nx * c->al[l].ny;
            return a >= (size_t)2048 * 2048 ? 0 : a >= (size_t)1024 * 1024 ? 32 : 16;
        }
        return v == 1 ? 16 : v == 2 ? 32 : 0;
    }
    template <typename F>
    static void with_edge(int tt, F&& f) {
        if (tt == 16)
            f(std::integral_constant<int, 16>{});
        else
            f(std::integral_constant<int, 32>{});
    }

    // Pass 1 and the coefficient solve of the s-step GMRES(MM) on level l (x0 = A.x if X0).
    template <int MM, bool X0>
    void sstep_gram_solve(int l, int S, int tt) {
        AdrLevel& A = c->al[l];
        constexpr int NG = (MM + 1) * (MM + 1);
        const double bytes = ((X0 ? 3 : 2) * sizeof(C) + 2 * sizeof(T)) * NN2(A.nx, A.ny);
        const C* x0 = X0 ? (const C*)A.x : nullptr;
        int ng = 0;
        if (tt) {
            with_edge(tt, [&](auto e) {
                constexpr int TT = decltype(e)::value;
                ng = Tile<MM, X0, true, TT>::tiles(A.nx, A.ny);
                REQUIRE((size_t)ng * NG <= c->partials_cap, "s-step: too many tiles for the reduction scratch");
                LAUNCH(c, bytes, (k_sstep_gram_tile<T, MM, X0, TT>), dim3(ng), dim3(BLOCK), st, A.A,
                       (const T*)A.px, (const T*)A.py, (const C*)A.c0, (const C*)A.b, x0, c->partials);
            });
        } else {
            ng = March<MM, X0, true>::units(A.nx, A.ny, S);
            REQUIRE((size_t)ng * NG <= c->partials_cap, "s-step: too many segments for the reduction scratch");
            LAUNCH(c, bytes, (k_sstep_gram<T, MM, X0>), dim3(ng), dim3(64), st, A.A, S, (const T*)A.px,
                   (const T*)A.py, (const C*)A.c0, (const C*)A.b, x0, c->partials);
        }
        LAUNCH(c, 8.0 * NG * ng, (k_sstep_solve<MM>), dim3(1), dim3(SOLVE_THREADS), st, (const double*)c->partials,
               ng, 1e-12, A.K);
    }

    // Pass 2 with the plain epilogue: xout = x0 + sum c_j K_{j-1} (x0 = A.x if X0).
    template <int MM, bool X0>
    void sstep_combine_x(int l, int S, int tt, C* xout) {
        AdrLevel& A = c->al[l];
        const double bytes = ((X0 ? 4 : 3) * sizeof(C) + 2 * sizeof(T)) * NN2(A.nx, A.ny);
        const C* x0 = X0 ? (const C*)A.x : nullptr;
        if (tt) {
            with_edge(tt, [&](auto e) {
                constexpr int TT = decltype(e)::value;
                LAUNCH(c, bytes, (k_sstep_combine_tile<T, MM, X0, TT>), dim3(Tile<MM, X0, false, TT>::tiles(A.nx, A.ny)),
                       dim3(BLOCK), st, A.A, (const T*)A.px, (const T*)A.py, (const C*)A.c0, (const C*)A.b, x0,
                       (const KrylovScal*)A.K, xout);
            });
        } else {
            LAUNCH(c, bytes, (k_sstep_combine<T, MM, X0, EPI_X>), dim3(March<MM, X0, false>::units(A.nx, A.ny, S)), dim3(64),
                   st, A.A, S, (const T*)A.px, (const T*)A.py, (const C*)A.c0, (const C*)A.b, x0,
                   (const KrylovScal*)A.K, xout, ModArgs<T>{});
        }
    }

    // s-step GMRES(MM) on ADR level l.
    template <int MM>
    void gmres_sstep(int l, bool x0_zero, int epi, const ModArgs<T>* ma) {
        AdrLevel& A = c->al[l];
        const int S = sstep_steps(l), tt = sstep_tile_edge(l);
        const double nn = NN2(A.nx, A.ny);
        if (x0_zero) {
            REQUIRE(epi == EPI_X, "fused ADR epilogue on a pre-smoother");
            sstep_gram_solve<MM, false>(l, S, tt);
            sstep_combine_x<MM, false>(l, S, tt, (C*)A.x);
            return;
        }
        sstep_gram_solve<MM, true>(l, S, tt);
        if (epi == EPI_X) {
            sstep_combine_x<MM, true>(l, S, tt, (C*)A.xalt);
            std::swap(A.x, A.xalt);
        } else if (epi == EPI_MOD) {
            const int nc = March<MM, true, false>::units(A.nx, A.ny, S);
            LAUNCH(c, (6 * sizeof(C) + 2 * sizeof(T)) * nn, (k_sstep_combine<T, MM, true, EPI_MOD>), dim3(nc),
                   dim3(64), st, A.A, S, (const T*)A.px, (const T*)A.py, (const C*)A.c0, (const C*)A.b,
                   (const C*)A.x, (const KrylovScal*)A.K, (C*)nullptr, *ma);
        } else if constexpr (MM <= 3) {
            const int nc = March<MM, true, false, 1>::units(A.nx, A.ny, S);
            LAUNCH(c, (8 * sizeof(C) + 3 * sizeof(T)) * nn, (k_sstep_combine<T, MM, true, EPI_MODRD>), dim3(nc),
                   dim3(64), st, A.A, S, (const T*)A.px, (const T*)A.py, (const C*)A.c0, (const C*)A.b,
                   (const C*)A.x, (const KrylovScal*)A.K, (C*)nullptr, *ma);
        } else {
            throw Error(HELM_EINVAL, "fused ADR epilogue needs gmres_m <= 3");
        }
    }

    // GMRES(m) smoother on ADR level l (x = A.x, b = A.b); epi != EPI_X (s-step form,
    // x0 != 0 only) hands the result to that epilogue instead of A.x.
    bool sstep_form(int m) const { return m <= 4 && !c->d.gmres_arnoldi; }
    void gmres(int l, int m, bool x0_zero, int epi = EPI_X, const ModArgs<T>* ma = nullptr) {
        // one workgroup on the coarsest level, s-step form on the larger ones
        if (l == c->LA && gmres_block(l, m, x0_zero)) return;
        if (sstep_form(m)) {
            switch (m) {
                case 1: gmres_sstep<1>(l, x0_zero, epi, ma); break;
                case 2: gmres_sstep<2>(l, x0_zero, epi, ma); break;
                case 3: gmres_sstep<3>(l, x0_zero, epi, ma); break;
                default: gmres_sstep<4>(l, x0_zero, epi, ma); break;
            }
            return;
        }
        REQUIRE(epi == EPI_X, "fused ADR epilogue without the s-step smoother");
        switch (nv_bucket(m)) {
            case 4: gmres_nv<4>(l, m, x0_zero); break;
            case 12: gmres_nv<12>(l, m, x0_zero); break;
            default: gmres_nv<MAXM>(l, m, x0_zero); break;
        }
    }
};

// ------------------------------------------------------------------ outer Krylov (host-driven Givens)
using cd = std::complex<double>;

static void givens(cd a, cd b, double& c, cd& s) {
    if (b == 0.0) {
        c = 1.0;
        s = 0.0;
        return;
    }
    if (a == 0.0) {
        c = 0.0;
        s = 1.0;
        return;
    }
    double rho = std::hypot(std::abs(a), std::abs(b));
    c = std::abs(a) / rho;
    s = (a / std::abs(a)) * std::conj(b) / rho;
}

// One restart cycle of FGMRES on the fine grid with vectors of precision P and a
// preconditioner that maps V_j to Z_j.  Returns iterations done; updates x (precision P)
// in place with x += Z y.  est_out: final residual estimate / gnorm.
template <typename P, typename Prec>
static int fgmres_cycle(helm_ctx c, hipStream_t st, const void* n2_fine, void** V, void** Z, KrylovScal* K,
                        bool z_scaled, void* x, double gnorm, double stop_abs, int maxit_left, Prec&& prec,
                        std::vector<double>* history, double* est_out, bool* breakdown) {
    using Cp = cplx<P>;
    const int m = c->d.restart;
    const Geom G = make_geom_sys(c);
    const size_t N = (size_t)G.nx * G.ny;
    // K init from V[0]
    const int nbf = c->tn.fgmres_blocks > 0 ? std::min(c->tn.fgmres_blocks, MAXRED) : flat_blocks(N, MAXRED);
    LAUNCH(c, sizeof(Cp) * double(N), (k_krylov_init_norm<P>), dim3(nbf), dim3(BLOCK), st, N, (const Cp*)V[0],
           c->partials);
    krylov_fin<MAXM>(c, st, nbf, FIN_INIT, 0, m, K, 0.0);
    KrylovScal hk;
    HIPCHK(hipMemcpyAsync(&hk.beta, &K->beta, sizeof(double), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    const double beta = hk.beta;
    *breakdown = false;
    if (!(beta > 0.0) || !std::isfinite(beta)) {
        *est_out = beta / gnorm;
        *breakdown = !std::isfinite(beta);
        return 0;
    }
    VecSet<P> Vs{}, Zs{};
    for (int i = 0; i <= m; ++i) Vs.v[i] = (const Cp*)V[i];
    for (int i = 0; i < m; ++i) Zs.v[i] = (const Cp*)Z[i];
    std::vector<std::vector<cd>> H(m + 1, std::vector<cd>(m, 0.0));
    std::vector<double> cs(m);
    std::vector<cd> sn(m), e(m + 1, 0.0);
    e[0] = beta;
    int used = 0;
    double est = beta / gnorm;
    // Iteration j + 1 is queued before the host reads the Hessenberg column of
    // iteration j, so the device never waits for the host's Givens update.  When the
    // host stops at column j, the queued iteration only touches state that the next
    // restart rewrites (its kernels exit early once the device marks a breakdown).
    const int jmax = std::min(m, maxit_left);
    const size_t cstride = 2 * (MAXM + 1);
    // Classical Gram-Schmidt twice with the second round lagging one pass: V[j] enters
    // iteration j after one round (V[0] = r0 needs none), z_j is the preconditioned
    // V[j], and the Arnoldi pass of iteration j applies the second round to V[j]
    // while it builds w = A z_j.  Every Hessenberg entry is the two-round one; the
    // subdiagonal H(j+1, j) that the host sees with column j comes from the norms
    // (||w||^2 - sum |d_i|^2) and is replaced on the device by the directly computed
    // norm one pass later.
    auto enqueue = [&](int j) {
        prec(j, K->zscale + j);  // Z[j] = preconditioned V[j] (scaled by zscale[j] if !z_scaled)
        static_for_host<MAXM>(j, [&](auto jc) {
            constexpr int J = decltype(jc)::value;
            LAUNCH(c, ((J + (J > 0 ? 4 : 3)) * sizeof(Cp) + sizeof(P)) * double(N), (k_fg_arnoldi<P, J>), dim3(nbf),
                   dim3(BLOCK), st, G, (const P*)n2_fine, (const Cp*)Z[J], z_scaled ? 0 : 1, Vs, (Cp*)V[J],
                   (Cp*)V[J + 1], (const KrylovScal*)K, c->partials);
            krylov_fin<MAXM>(c, st, nbf, FIN_LMV, J, m, K, 0.0);
            LAUNCH(c, (J + 3) * sizeof(Cp) * double(N), (k_fg_orth<P, J>), dim3(nbf), dim3(BLOCK), st, N, Vs,
                   (Cp*)V[J + 1], (const KrylovScal*)K, c->partials);
            krylov_fin<MAXM>(c, st, nbf, FIN_LORTH, J, m, K, 0.0);
        });
        HIPCHK(hipMemcpyAsync(c->hcol + j * cstride, K->H + 2 * (j * (MAXM + 1)), sizeof(double) * 2 * (j + 2),
                              hipMemcpyDeviceToHost, st));
        HIPCHK(hipEventRecord(c->col_ev[j], st));
    };
    if (jmax > 0) enqueue(0);
    for (int j = 0; j < jmax; ++j) {
        if (j + 1 < jmax) enqueue(j + 1);
        HIPCHK(hipEventSynchronize(c->col_ev[j]));
        const double* col = c->hcol + j * cstride;
        for (int i = 0; i <= j + 1; ++i) H[i][j] = cd(col[2 * i], col[2 * i + 1]);
        const double hn = col[2 * (j + 1)];
        for (int i = 0; i < j; ++i) {
            cd t1 = cs[i] * H[i][j] + sn[i] * H[i + 1][j];
            cd t2 = -std::conj(sn[i]) * H[i][j] + cs[i] * H[i + 1][j];
            H[i][j] = t1;
            H[i + 1][j] = t2;
        }
        givens(H[j][j], H[j + 1][j], cs[j], sn[j]);
        H[j][j] = cs[j] * H[j][j] + sn[j] * H[j + 1][j];
        H[j + 1][j] = 0.0;
        e[j + 1] = -std::conj(sn[j]) * e[j];
        e[j] = cs[j] * e[j];
        used = j + 1;
        est = std::abs(e[j + 1]) / gnorm;
        if (history) history->push_back(est);
        if (!std::isfinite(hn) || !std::isfinite(est)) {
            *breakdown = true;
            break;
        }
        if (std::abs(e[j + 1]) < stop_abs || hn == 0.0) break;
    }
    // y from the device Hessenberg (exact subdiagonals wherever the next Arnoldi pass
    // has run); x += sum y_i s_i Z_i with the factors the preconditioner inputs had
    if (used > 0) {
        LAUNCH(c, 0.0, k_fgmres_lsq, dim3(1), dim3(64), st, K, used);
        LAUNCH(c, (used + 2) * sizeof(Cp) * double(N), (k_krylov_combine<P, MAXM>), dim3(flat_blocks(N)), dim3(BLOCK),
               st, N, Zs, (const KrylovScal*)K, (const Cp*)x, (Cp*)x, z_scaled ? 2 : 1);
    }
    HIPCHK(hipStreamSynchronize(st));
    *est_out = est;
    return used;
}

// Iterative refinement: an inner FP32 FGMRES run stops once its residual estimate
// predicts the outer tolerance with this margin (max(1e-4, REFINE_MARGIN tol ||g|| / ||r||)
// relative to its right-hand side r / ||r||), or after one restart cycle; the FP64
// residual then decides.  The margin covers the gap between the FP32 estimate and the
// FP64 residual; a miss costs one more short inner run.
constexpr double REFINE_MARGIN = 0.9;

static void residual_fp64(helm_ctx c, hipStream_t st, const void* g, const void* u, void* r, double* rn, double* gn) {
    const Geom G = make_geom_sys(c);
    const int nbt = red_blocks(G.nx, G.ny);
    LAUNCH(c, (3 * 16.0 + 8.0 + (r ? 16.0 : 0.0)) * NN2(G.nx, G.ny), k_residual_norms, dim3(nbt), tile_block(), st, G,
           (const double*)c->n2f, (const c128*)g, (const c128*)u, (c128*)r, c->partials);
    LAUNCH(c, 16.0 * nbt, (k_finalize_sums<2>), dim3(1), dim3(FBLOCK), st, (const double*)c->partials, nbt, 2,
           c->dscal);
    double h[2];
    HIPCHK(hipMemcpyAsync(h, c->dscal, sizeof(h), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    if (rn) *rn = std::sqrt(h[0]);
    if (gn) *gn = std::sqrt(h[1]);
}

static void drop_graphs(helm_ctx c);

// Chebyshev coefficients of every level for the pre, post and coarsest step counts (the
// three-term recurrence of eq. cheb on [lambda_l / alpha_l, lambda_l]) and the per-level
// (lambda, alpha), written to the context's device table.
static void write_cycle_tables(helm_ctx c) {
    CycleDev h{};
    const int ms[3] = {c->d.cheb_pre, c->d.cheb_post, c->d.cheb_coarse};
    h.la[0] = c->w[0];
    for (int l = 2; l <= c->L; ++l) {
        const double lam = c->wl[l].lam, alpha = c->w[l - 1];
        h.la[2 * l] = lam;
        h.la[2 * l + 1] = alpha;
        const double a = lam / alpha;
        const double theta = 0.5 * (lam + a);
        const double dc = 0.5 * (lam - a);
        for (int kind = 0; kind < 3; ++kind) {
            double* t = h.cheb[l][kind];
            t[0] = double(1.0 / theta);
            double rho = dc / theta;
            for (int step = 1; step < ms[kind] && step < CHEB_ROWS; ++step) {
                const double den = 2.0 * theta - dc * rho;
                const double rho_new = dc / den;
                t[3 * step + 1] = rho_new * rho;
                t[3 * step + 2] = 2.0 / den;
                rho = rho_new;
            }
        }
    }
    HIPCHK(hipMemcpy(c->cdev, &h, sizeof(h), hipMemcpyHostToDevice));
}

// ------------------------------------------------------------------ setup
// The descriptor a context keeps: ny = n for a square grid given with ny = 0.
static helm_desc desc_normalized(const helm_desc& d) {
    helm_desc o = d;
    if (o.ny == 0) o.ny = o.n;
    return o;
}

static void validate(const helm_desc* d) {
    REQUIRE(d != nullptr, "desc is NULL");
    REQUIRE(d->n >= 16 && d->n <= 8192 && (d->n & (d->n - 1)) == 0, "n must be a power of two in [16, 8192]");
    const int ny = d->ny ? d->ny : d->n;
    REQUIRE(ny >= 16 && ny <= 8192 && (ny & (ny - 1)) == 0, "ny must be 0 or a power of two in [16, 8192]");
    REQUIRE(ny <= 16 * d->n && d->n <= 16 * ny, "n and ny may differ by a factor of 16 at most");
    int lg = 0;
    while ((1 << lg) < std::min(d->n, ny)) ++lg;
    REQUIRE(d->levels >= 2 && d->levels <= lg - 1, "levels must be in [2, log2(min(n, ny)) - 1]");
    REQUIRE(d->k > 0 && std::isfinite(d->k), "k must be positive");
    REQUIRE(d->damping_cells >= 1, "damping_cells must be >= 1");
    REQUIRE(d->damping_strength >= 0 && std::isfinite(d->damping_strength), "damping_strength must be >= 0");
    REQUIRE(d->shift >= 0 && std::isfinite(d->shift), "shift must be >= 0");
    REQUIRE(d->cycle_shift >= 0 && std::isfinite(d->cycle_shift), "cycle_shift must be >= 0");
    REQUIRE(d->sign == 1 || d->sign == -1, "sign must be +1 or -1");
    REQUIRE(d->cycle_prec == HELM_C64 || d->cycle_prec == HELM_C128, "cycle_prec must be HELM_C64 or HELM_C128");
    REQUIRE(d->adr_steps >= 0 && d->adr_steps <= 64, "adr_steps must be in [0, 64]");
    REQUIRE(d->cheb_pre >= 1 && d->cheb_post >= 1 && d->cheb_coarse >= 1 && d->cheb_pre <= 64 &&
                d->cheb_post <= 64 && d->cheb_coarse <= 64,
            "Chebyshev step counts must be in [1, 64]");
    REQUIRE(d->gmres_m >= 1 && d->gmres_m <= MAXM && d->gmres_coarse_m >= 1 && d->gmres_coarse_m <= MAXM,
            "GMRES dimensions must be in [1, 24]");
    REQUIRE(d->restart >= 1 && d->restart <= MAXM, "restart must be in [1, 24]");
    REQUIRE(d->gmres_arnoldi == 0 || d->gmres_arnoldi == 1, "gmres_arnoldi must be 0 or 1");
    REQUIRE(d->use_graphs == 0 || d->use_graphs == 1, "use_graphs must be 0 or 1");
    REQUIRE(d->tail_n >= 0, "tail_n must be >= 0");
    REQUIRE(d->wave_tail_n >= 0, "wave_tail_n must be >= 0");
    REQUIRE(d->adr_levels >= 0, "adr_levels must be >= 0");
}

static void build(helm_ctx c, const double* velocity, hipStream_t st) {
    const helm_desc& d = c->d;
    const int n = d.n, L = d.levels;
    c->L = L;
    c->LA = d.adr_levels > 0 ? std::min(L, 1 + d.adr_levels) : L;
    c->f32 = d.cycle_prec == HELM_C64;
    const bool f64c = !c->f32;
    const size_t NF = (size_t)n * d.ny;
    // reduction scratch: enough partials for any tiled kernel on the fine grid
    const size_t maxblk = std::max<size_t>((size_t)tiles_of(n, d.ny), 2048);
    c->partials_cap = maxblk * std::max(2 * MAXM + 4, (GMAX + 1) * (GMAX + 2));
    c->partials = (double*)dalloc(c, c->partials_cap * sizeof(double));
    c->dscal = (double*)dalloc(c, 64 * sizeof(double));
    c->Kout = (KrylovScal*)dalloc(c, sizeof(KrylovScal));
    c->Kin = (KrylovScal*)dalloc(c, sizeof(KrylovScal));
    HIPCHK(hipMemsetAsync(c->Kout, 0, sizeof(KrylovScal), st));
    HIPCHK(hipMemsetAsync(c->Kin, 0, sizeof(KrylovScal), st));
    // fine n^2 in FP64, velocity check
    c->n2f = (double*)dalloc(c, NF * sizeof(double));
    int* bad = (int*)c->dscal;
    HIPCHK(hipMemsetAsync(bad, 0, sizeof(int), st));
    hipLaunchKernelGGL(k_slowness2, dim3(flat_blocks(NF)), dim3(BLOCK), 0, st, NF, velocity, c->n2f, bad);
    HIPCHK(hipGetLastError());
    int hbad = 0;
    HIPCHK(hipMemcpyAsync(&hbad, bad, sizeof(int), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    REQUIRE(hbad == 0, "velocity must be positive and finite everywhere");
    // wave levels
    c->wl.assign(L + 1, WaveLevel{});
    for (int l = 1; l <= L; ++l) {
        WaveLevel& W = c->wl[l];
        W.nx = lnx(c, l);
        W.ny = lny(c, l);
        W.G = make_geom(c, l);
        W.f64 = f64c || l == L;
        const size_t Nl = (size_t)W.nx * W.ny;
        if (l == 1 && W.f64) {
            W.n2 = c->n2f;
        } else {
            W.n2 = dalloc(c, Nl * rsize(W.f64));
            if (W.f64)
                hipLaunchKernelGGL((k_inject_real<double, double>), dim3(flat_blocks(Nl)), dim3(BLOCK), 0, st, W.nx,
                                   W.ny, 1 << (l - 1), n, (const double*)c->n2f, (double*)W.n2);
            else
                hipLaunchKernelGGL((k_inject_real<float, double>), dim3(flat_blocks(Nl)), dim3(BLOCK), 0, st, W.nx,
                                   W.ny, 1 << (l - 1), n, (const double*)c->n2f, (float*)W.n2);
        }
        if (l >= 2) {
            W.g = dalloc(c, Nl * csize(W.f64));
            W.u = dalloc(c, Nl * csize(W.f64));
            W.t = dalloc(c, Nl * csize(W.f64));
            W.r = dalloc(c, Nl * csize(W.f64));
            W.d = dalloc(c, Nl * csize(W.f64));
        }
        // statistics from the FP64 fine field by injection (through a FP64 copy on coarse levels)
        const double* n2d = c->n2f;
        double* tmp = nullptr;
        if (l > 1) {
            HIPCHK(hipMalloc((void**)&tmp, Nl * sizeof(double)));
            hipLaunchKernelGGL((k_inject_real<double, double>), dim3(flat_blocks(Nl)), dim3(BLOCK), 0, st, W.nx,
                               W.ny, 1 << (l - 1), n, (const double*)c->n2f, tmp);
            n2d = tmp;
        }
        const int nbs = flat_blocks(Nl, 1024);
        hipLaunchKernelGGL(k_level_stats, dim3(nbs), dim3(BLOCK), 0, st, W.G, n2d, c->partials);
        std::vector<double> ps(3 * (size_t)nbs);
        HIPCHK(hipMemcpyAsync(ps.data(), c->partials, ps.size() * sizeof(double), hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
        double hs[3] = {0.0, 0.0, 0.0};
        for (int q = 0; q < nbs; ++q) {
            hs[0] = std::max(hs[0], ps[3 * q]);
            hs[1] = std::max(hs[1], ps[3 * q + 1]);
            hs[2] += ps[3 * q + 2];
        }
        W.lam = (hs[0] + 4.0 * W.G.inv_h2) * (hs[0] + 4.0 * W.G.inv_h2);
        W.n2max = hs[1];
        W.n2mean = hs[2] / double((size_t)(W.nx - 1) * (W.ny - 1));
        if (tmp) {
            HIPCHK(hipFree(tmp));
        }
    }
    // first level (>= 3) small enough for the one-workgroup tail of the wave cycle
    c->LT = 0;
    for (int l = 3; l <= L && l <= WT_MAXL; ++l)
        if (std::max(c->wl[l].nx, c->wl[l].ny) <= d.wave_tail_n) {
            c->LT = l;
            break;
        }
    // default weights
    c->w.assign(L, 0.0);
    {
        const double h1 = 1.0 / inv_h(c, 1);
        const double K = d.k * d.k * c->wl[1].n2max * h1 * h1;
        c->w[0] = (4.0 - K) / (5.0 - K);
        for (int l = 2; l <= L; ++l)
            c->w[l - 1] = median_alpha(d.k, c->wl[l].n2mean, c->wl[l].nx, c->wl[l].ny, 1.0 / inv_h(c, l),
                                       c->wl[l].lam);
    }
    c->w_default = c->w;
    c->cdev = (CycleDev*)dalloc(c, sizeof(CycleDev));
    write_cycle_tables(c);
    // level-1 second iterate
    c->ws1 = dalloc(c, NF * csize(f64c));
    // ADR levels
    c->al.assign(L + 1, AdrLevel{});
    if (L >= 3) {
        for (int l = 2; l <= c->LA; ++l) {
            AdrLevel& A = c->al[l];
            A.nx = lnx(c, l);
            A.ny = lny(c, l);
            A.A = make_adr_geom(c, l);
            const size_t Nl = (size_t)A.nx * A.ny;
            A.px = dalloc(c, Nl * rsize(f64c));
            A.py = dalloc(c, Nl * rsize(f64c));
            A.c0 = dalloc(c, Nl * csize(f64c));
            A.b = dalloc(c, Nl * csize(f64c));
            A.x = dalloc(c, Nl * csize(f64c));
            A.xalt = dalloc(c, Nl * csize(f64c));
            const int m = (l == c->LA) ? d.gmres_coarse_m : d.gmres_m;
            char* vb = (char*)dalloc(c, (size_t)(m + 1) * Nl * csize(f64c));  // V_0..V_m contiguous
            for (int i = 0; i <= m; ++i) A.V[i] = vb + (size_t)i * Nl * csize(f64c);
            A.K = (KrylovScal*)dalloc(c, sizeof(KrylovScal));
            HIPCHK(hipMemsetAsync(A.K, 0, sizeof(KrylovScal), st));
            if (l == 2) A.balt = dalloc(c, Nl * csize(f64c));
        }
        c->wl[2].ualt = dalloc(c, (size_t)c->wl[2].nx * c->wl[2].ny * csize(c->wl[2].f64));
        c->car2 = dalloc(c, (size_t)c->wl[2].nx * c->wl[2].ny * csize(f64c));
        helm_ctx_s::PhaseSet s0{};
        for (int l = 2; l <= c->LA; ++l) {
            s0.px[l] = c->al[l].px;
            s0.py[l] = c->al[l].py;
            s0.c0[l] = c->al[l].c0;
        }
        s0.car = c->car2;
        c->sets.assign(1, s0);
    }
    // FP64 residual vectors; the Krylov bases of the outer solvers are allocated by
    // the first solve in each mode (ensure_solver_ws)
    c->fV[0] = dalloc(c, NF * sizeof(c128));
    c->rbuf = dalloc(c, NF * sizeof(c128));
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(st));
}

// Points the ADR levels and the level-2 carrier at phase set m.
static void use_set(helm_ctx c, int m) {
    const helm_ctx_s::PhaseSet& S = c->sets[m];
    for (int l = 2; l <= c->LA; ++l) {
        c->al[l].px = S.px[l];
        c->al[l].py = S.py[l];
        c->al[l].c0 = S.c0[l];
    }
    c->car2 = S.car;
}

// ADR coefficients of every ADR level and the level-2 carrier from the fine phase phi,
// into the current phase set.
static void build_phase(helm_ctx c, const void* phi, int is64, hipStream_t st) {
    for (int l = 2; l <= c->LA; ++l) {
        AdrLevel& A = c->al[l];
        const Geom G = make_geom(c, l);
        const size_t Nl = (size_t)A.nx * A.ny;
        void* th = (l == 2) ? c->car2 : nullptr;
        const int nb = flat_blocks(Nl);
        if (c->f32) {
            if (is64)
                hipLaunchKernelGGL((k_adr_coef<float, double>), dim3(nb), dim3(BLOCK), 0, st, G, (const double*)c->n2f,
                                   (const double*)phi, c->d.k, c->d.sign, c->d.damping_strength, (float*)A.px,
                                   (float*)A.py, (c64*)A.c0, (c64*)th);
            else
                hipLaunchKernelGGL((k_adr_coef<float, float>), dim3(nb), dim3(BLOCK), 0, st, G, (const double*)c->n2f,
                                   (const float*)phi, c->d.k, c->d.sign, c->d.damping_strength, (float*)A.px,
                                   (float*)A.py, (c64*)A.c0, (c64*)th);
        } else {
            if (is64)
                hipLaunchKernelGGL((k_adr_coef<double, double>), dim3(nb), dim3(BLOCK), 0, st, G,
                                   (const double*)c->n2f, (const double*)phi, c->d.k, c->d.sign,
                                   c->d.damping_strength, (double*)A.px, (double*)A.py, (c128*)A.c0, (c128*)th);
            else
                hipLaunchKernelGGL((k_adr_coef<double, float>), dim3(nb), dim3(BLOCK), 0, st, G,
                                   (const double*)c->n2f, (const float*)phi, c->d.k, c->d.sign,
                                   c->d.damping_strength, (double*)A.px, (double*)A.py, (c128*)A.c0, (c128*)th);
        }
    }
    HIPCHK(hipGetLastError());
}

static void set_phase(helm_ctx c, const void* phi, int is64, hipStream_t st) {
    if (c->L < 3) {
        c->phase_set = true;
        ++c->data_gen;
        return;
    }
    use_set(c, 0);
    c->nsets = 1;
    build_phase(c, phi, is64, st);
    HIPCHK(hipStreamSynchronize(st));
    drop_graphs(c);
    c->phase_set = true;
    c->phase_factored = false;
    ++c->data_gen;
}

// Wave-Ray phases: count plane waves phi_m = nbar (cos theta_m x + sin theta_m y),
// theta_m = 2 pi m / count, nbar^2 the mean of n^2 over the fine unknowns.
static void set_rays(helm_ctx c, int count, hipStream_t st) {
    REQUIRE(count >= 1 && count <= 64, "helm_set_rays: count must be in 1..64");
    if (c->L < 3) {
        c->phase_set = true;
        ++c->data_gen;
        return;
    }
    const bool f64c = !c->f32;
    while ((int)c->sets.size() < count) {
        helm_ctx_s::PhaseSet S{};
        for (int l = 2; l <= c->LA; ++l) {
            const size_t Nl = (size_t)c->al[l].nx * c->al[l].ny;
            S.px[l] = dalloc(c, Nl * rsize(f64c));
            S.py[l] = dalloc(c, Nl * rsize(f64c));
            S.c0[l] = dalloc(c, Nl * csize(f64c));
        }
        const size_t N2 = (size_t)c->al[2].nx * c->al[2].ny;
        S.car = dalloc(c, N2 * csize(f64c));
        c->sets.push_back(S);
    }
    const int n = c->d.n;
    const size_t NF = (size_t)n * c->d.ny;
    double* phi = nullptr;
    HIPCHK(hipMalloc((void**)&phi, NF * sizeof(double)));
    const double nbar = std::sqrt(c->wl[1].n2mean);
    try {
        for (int m = 0; m < count; ++m) {
            const double th = 2.0 * M_PI * double(m) / double(count);
            hipLaunchKernelGGL(k_ray_phase, dim3(flat_blocks(NF)), dim3(BLOCK), 0, st, n, c->d.ny, nbar, std::cos(th),
                               std::sin(th), phi);
            use_set(c, m);
            build_phase(c, phi, 1, st);
        }
        HIPCHK(hipStreamSynchronize(st));
    } catch (...) {
        (void)hipStreamSynchronize(st);
        (void)hipFree(phi);
        use_set(c, 0);
        throw;
    }
    HIPCHK(hipFree(phi));
    use_set(c, 0);
    c->nsets = count;
    drop_graphs(c);
    c->phase_set = true;
    c->phase_factored = false;
    ++c->data_gen;
}

template <typename T>
static void run_cycle(helm_ctx c, const void* g, const void* u_in, void* u_out, hipStream_t st) {
    Engine<T> E(c, st);
    E.cycle(g, u_in, u_out);
}

static void cycle_eager(helm_ctx c, const void* g, const void* u_in, void* u_out, hipStream_t st) {
    if (c->f32)
        run_cycle<float>(c, g, u_in, u_out, st);
    else
        run_cycle<double>(c, g, u_in, u_out, st);
}

static void drop_graphs(helm_ctx c) {
    for (auto& e : c->graphs) (void)hipGraphExecDestroy(e.exec);
    c->graphs.clear();
    for (auto& a : c->adj_graph) {
        if (a.exec) (void)hipGraphExecDestroy(a.exec);
        a = helm::AdjGraph{};
    }
}

// One cycle: replays the graph captured for these pointers (capturing it on first
// use), or launches eagerly when graphs are off or per-launch profiling is on.
// The cycle's kernel arguments depend only on the pointers and the weights, so a
// graph stays valid until the weights change (drop_graphs).
static void cycle_any(helm_ctx c, const void* g, const void* u_in, void* u_out, hipStream_t st) {
    if (!c->d.use_graphs || c->prof.on) {
        cycle_eager(c, g, u_in, u_out, st);
        return;
    }
    for (auto& e : c->graphs) {
        if (e.g == g && e.uin == u_in && e.uout == u_out) {
            HIPCHK(hipGraphLaunch(e.exec, st));
            return;
        }
    }
    if (c->graphs.size() >= 64) drop_graphs(c);
    if (!c->cap_stream) HIPCHK(hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking));
    hipGraph_t graph = nullptr;
    HIPCHK(hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal));
    try {
        cycle_eager(c, g, u_in, u_out, c->cap_stream);
    } catch (...) {
        (void)hipStreamEndCapture(c->cap_stream, &graph);
        if (graph) (void)hipGraphDestroy(graph);
        throw;
    }
    HIPCHK(hipStreamEndCapture(c->cap_stream, &graph));
    hipGraphExec_t exec = nullptr;
    hipError_t e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    HIPCHK(e);
    c->graphs.push_back({g, u_in, u_out, exec});
    HIPCHK(hipGraphLaunch(exec, st));
}

// ------------------------------------------------------------------ solve
// Krylov bases of the outer solver of `mode` (first use only): mode 0 keeps
// restart+1 V and restart Z vectors in complex128 (plus complex64 staging for
// complex64 cycles), mode 1 the complex64 inner bases and correction.
static void ensure_solver_ws(helm_ctx c, int mode) {
    const size_t NF = (size_t)c->d.n * c->d.ny;
    const int m = c->d.restart;
    if (!c->hcol) {
        HIPCHK(hipHostMalloc((void**)&c->hcol, sizeof(double) * MAXM * 2 * (MAXM + 1), hipHostMallocDefault));
        for (int i = 0; i < MAXM; ++i) HIPCHK(hipEventCreateWithFlags(&c->col_ev[i], hipEventDisableTiming));
    }
    if (mode == 0 && !c->fZ[0]) {
        for (int i = 1; i <= m; ++i) c->fV[i] = dalloc(c, NF * sizeof(c128));
        for (int i = 0; i < m; ++i) c->fZ[i] = dalloc(c, NF * sizeof(c128));
        if (c->f32) {
            c->cyc_g = dalloc(c, NF * sizeof(c64));
            c->cyc_u = dalloc(c, NF * sizeof(c64));
        }
    }
    if (mode == 1 && !c->iV[0]) {
        for (int i = 0; i <= m; ++i) c->iV[i] = dalloc(c, NF * sizeof(c64));
        for (int i = 0; i < m; ++i) c->iZ[i] = dalloc(c, NF * sizeof(c64));
        c->dbuf = dalloc(c, NF * sizeof(c64));
    }
}

static helm_status solve(helm_ctx c, const void* g, void* u, double tol, int maxit, int mode, int* iters,
                         double* relres, double* history, hipStream_t st) {
    const size_t NF = (size_t)c->d.n * c->d.ny;
    if (mode == 1) REQUIRE(c->f32, "mode 1 (iterative refinement) needs cycle_prec = HELM_C64");
    ensure_solver_ws(c, mode);
    double rn = 0, gn = 0;
    residual_fp64(c, st, g, u, c->fV[0], &rn, &gn);
    std::vector<double> hist;
    int its = 0;
    if (!std::isfinite(gn) || !std::isfinite(rn)) {
        // NaN or Inf in g or in the initial iterate: nothing is iterated, u is left as given
        *iters = 0;
        *relres = rn / gn;
        return HELM_EBREAKDOWN;
    }
    if (!(gn > 0.0)) {
        LAUNCH(c, 16.0 * double(NF), (k_zero<double>), dim3(flat_blocks(NF)), dim3(BLOCK), st, NF, (c128*)u);
        HIPCHK(hipStreamSynchronize(st));
        *iters = 0;
        *relres = 0.0;
        return HELM_OK;
    }
    const double r0 = rn;
    helm_status status = HELM_OK;
    bool converged = rn / gn < tol;
    if (mode == 0) {
        while (!converged && its < maxit) {
            double est = 0;
            bool bd = false;
            auto prec = [&](int j, const double* ds) {
                if (c->f32) {
                    LAUNCH(c, 24.0 * double(NF), (k_cast_scale_dev<float, double>), dim3(flat_blocks(NF)), dim3(BLOCK),
                           st, NF, (const c128*)c->fV[j], (c64*)c->cyc_g, ds);
                    cycle_any(c, c->cyc_g, nullptr, c->cyc_u, st);
                    LAUNCH(c, 24.0 * double(NF), (k_cast_scale<double, float>), dim3(flat_blocks(NF)), dim3(BLOCK), st, NF,
                                       (const c64*)c->cyc_u, (c128*)c->fZ[j], 1.0);
                } else {
                    cycle_any(c, c->fV[j], nullptr, c->fZ[j], st);
                }
            };
            // Z scaled by 1/||V_j|| already when the cycle input was normalised (complex64 path)
            const bool zs = c->f32;
            int used = fgmres_cycle<double>(c, st, c->n2f, c->fV, c->fZ, c->Kout, zs, u, gn, tol * gn, maxit - its,
                                            prec, &hist, &est, &bd);
            its += used;
            residual_fp64(c, st, g, u, c->fV[0], &rn, &gn);
            if (bd || !std::isfinite(rn) || rn > 1e4 * r0) {
                status = HELM_EBREAKDOWN;
                break;
            }
            converged = rn / gn < tol;
            if (used == 0) break;
        }
    } else {
        REQUIRE(c->f32, "mode 1 (iterative refinement) needs cycle_prec = HELM_C64");
        const double eta = 1e-4;
        while (!converged && its < maxit) {
            // inner right-hand side r / ||r|| in complex64 (fV[0] holds r)
            LAUNCH(c, 0.0, k_norm_scales, dim3(1), dim3(64), st, c->dscal);
            LAUNCH(c, 24.0 * double(NF), (k_cast_scale_dev<float, double>), dim3(flat_blocks(NF)), dim3(BLOCK), st, NF,
                   (const c128*)c->fV[0], (c64*)c->iV[0], (const double*)c->dscal + 2);
            LAUNCH(c, 8.0 * double(NF), (k_zero<float>), dim3(flat_blocks(NF)), dim3(BLOCK), st, NF, (c64*)c->dbuf);
            auto prec = [&](int j, const double*) { cycle_any(c, c->iV[j], nullptr, c->iZ[j], st); };
            double est = 0;
            bool bd = false;
            const double target = std::max(eta, REFINE_MARGIN * tol * gn / rn);
            int used = fgmres_cycle<float>(c, st, c->wl[1].n2, c->iV, c->iZ, c->Kin, false, c->dbuf, 1.0, target,
                                           maxit - its, prec, nullptr, &est, &bd);
            its += used;
            LAUNCH(c, 40.0 * double(NF), (k_add_cast_dev<double, float>), dim3(flat_blocks(NF)), dim3(BLOCK), st, NF,
                   (const c64*)c->dbuf, (c128*)u, (const double*)c->dscal + 3);
            residual_fp64(c, st, g, u, c->fV[0], &rn, &gn);
            hist.push_back(rn / gn);
            if (bd || !std::isfinite(rn) || rn > 1e4 * r0) {
                status = HELM_EBREAKDOWN;
                break;
            }
            converged = rn / gn < tol;
            if (used == 0) break;
        }
    }
    *iters = its;
    *relres = rn / gn;
    if (history)
        for (size_t i = 0; i < hist.size() && i < (size_t)maxit + 1; ++i) history[i] = hist[i];
    if (status == HELM_OK && !converged) status = HELM_ENOCONV;
    return status;
}

#include "eik_host.hpp"
#include "adjoint_host.hpp"
#include "batch.hpp"
#include "tune.hpp"

// ------------------------------------------------------------------ allocation-free residual
// helm_residual_noalloc keeps its reduction scratch in this file-scope device array
// instead of the context's workspace: the per-block partial sums of ||r||^2 and ||g||^2
// (two doubles for each of at most MAXRED blocks), then the two totals.  Each GPU holds
// its own copy for the life of the process.  In host code the name `scratch` is only a
// host-side handle; the device address comes from hipGetSymbolAddress, resolved once per
// device (helm_setup, or the first call on a device) and kept in g_scratch_dev.
constexpr size_t NOALLOC_PARTIALS = 2 * (size_t)MAXRED;
constexpr size_t NOALLOC_DOUBLES = NOALLOC_PARTIALS + 32;
static __device__ __align__(256) double scratch[NOALLOC_DOUBLES];
constexpr int NOALLOC_MAX_DEVICES = 64;
static std::mutex g_scratch_mu;
static double* g_scratch_dev[NOALLOC_MAX_DEVICES] = {};

// Device address of `scratch` on the current device.
static double* noalloc_scratch() {
    int dev = 0;
    HIPCHK(hipGetDevice(&dev));
    if (dev < 0 || dev >= NOALLOC_MAX_DEVICES)
        throw Error(HELM_EINVAL, "device ordinal " + std::to_string(dev) + " beyond the static scratch table");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_dev[dev]) {
        void* p = nullptr;
        HIPCHK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) throw Error(HELM_EHIP, "hipGetSymbolAddress returned a null address for the residual scratch");
        g_scratch_dev[dev] = (double*)p;
    }
    return g_scratch_dev[dev];
}

// FP64 residual and norms of residual_fp64 with the reduction in `scratch`: no
// allocation, no event, no graph; the same kernels in the same order, so the results
// equal helm_residual's bit for bit.
static void residual_fp64_noalloc(helm_ctx c, hipStream_t st, const void* g, const void* u, void* r, double* rn,
                                  double* gn) {
    const Geom G = make_geom_sys(c);
    const int nbt = red_blocks(G.nx, G.ny);
    if ((size_t)2 * nbt > NOALLOC_PARTIALS)
        throw Error(HELM_EINVAL, "helm_residual_noalloc: " + std::to_string(nbt) + " reduction blocks exceed the " +
                                     std::to_string(NOALLOC_PARTIALS / 2) + " of the static scratch");
    double* sp = noalloc_scratch();
    hipLaunchKernelGGL(k_residual_norms, dim3(nbt), tile_block(), 0, st, G, (const double*)c->n2f, (const c128*)g,
                       (const c128*)u, (c128*)r, sp, BatchIdx{});
    hipLaunchKernelGGL((k_finalize_sums<2>), dim3(1), dim3(FBLOCK), 0, st, (const double*)sp, nbt, 2,
                       sp + NOALLOC_PARTIALS, BatchIdx{});
    HIPCHK(hipGetLastError());
    double h[2];
    HIPCHK(hipMemcpyAsync(h, sp + NOALLOC_PARTIALS, sizeof(h), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    if (rn) *rn = std::sqrt(h[0]);
    if (gn) *gn = std::sqrt(h[1]);
}

}  // namespace helm

// ================================================================== C ABI
using namespace helm;

static helm_status fail(const Error& e) {
    g_last_error = e.what();
    return e.code;
}

#define ABI_GUARD(...)                                             \
    try {                                                          \
        __VA_ARGS__                                                \
    } catch (const Error& e) {                                     \
        return fail(e);                                            \
    } catch (const std::exception& e) {                            \
        g_last_error = e.what();                                   \
        return HELM_EHIP;                                          \
    } catch (...) {                                                \
        g_last_error = "unknown error";                            \
        return HELM_EHIP;                                          \
    }

extern "C" {

void helm_desc_default(helm_desc* d, int32_t n, double k) {
    if (!d) return;
    std::memset(d, 0, sizeof(*d));
    d->n = n;
    int lg = 0;
    while (lg < 31 && (1 << lg) < n) ++lg;
    int L = std::min(7, lg - 3);
    d->levels = L < 2 ? 2 : L;
    d->k = k;
    d->damping_cells = 16;
    d->damping_strength = 0.5;
    d->sign = 1;
    d->cycle_prec = HELM_C128;
    d->adr_steps = 8;
    d->cheb_pre = 5;
    d->cheb_post = 5;
    d->cheb_coarse = 10;
    d->gmres_m = 3;
    d->gmres_coarse_m = 3;
    d->level3_literal = 0;
    d->restart = 20;
    d->gmres_arnoldi = 0;
    d->use_graphs = 1;
    d->tail_n = 64;
    d->wave_tail_n = 32;
    d->adr_levels = 3;
    d->shift = 0.0;
    d->cycle_shift = 0.0;
}

helm_status helm_setup(const helm_desc* desc, const double* velocity, helm_ctx* out, void* stream) {
    ABI_GUARD({
        REQUIRE(out != nullptr, "out is NULL");
        validate(desc);
        REQUIRE(velocity != nullptr, "velocity is NULL");
        helm_ctx c = new helm_ctx_s();
        c->d = desc_normalized(*desc);
        try {
            build(c, velocity, (hipStream_t)stream);
            (void)noalloc_scratch();
        } catch (...) {
            helm_destroy(c);
            throw;
        }
        *out = c;
        return HELM_OK;
    })
}

helm_status helm_set_phase(helm_ctx ctx, const void* phi, int32_t phi_is_f64, void* stream) {
    ABI_GUARD({
        REQUIRE(ctx != nullptr && phi != nullptr, "NULL argument");
        set_phase(ctx, phi, phi_is_f64 != 0, (hipStream_t)stream);
        return HELM_OK;
    })
}

helm_status helm_set_rays(helm_ctx ctx, int32_t count, void* stream) {
    ABI_GUARD({
        REQUIRE(ctx != nullptr, "NULL argument");
        set_rays(ctx, count, (hipStream_t)stream);
        return HELM_OK;
    })
}

helm_status helm_eikonal(helm_ctx ctx, const double* src_xy, int32_t nsrc, int32_t max_rounds, double tol,
                         void* tau1_out, void* phi_out, int32_t* rounds, double* change, void* stream) {
    ABI_GUARD({
        REQUIRE(ctx != nullptr, "NULL argument");
        int r = 0;
        double ch = 0.0;
        const helm_status st = eikonal(ctx, src_xy, nsrc, max_rounds, tol, tau1_out, phi_out, &r, &ch,
                                       (hipStream_t)stream);
        if (rounds) *rounds = r;
        if (change) *change = ch;
        return st;
    })
}

helm_status helm_set_weights(helm_ctx ctx, const double* w) {
    ABI_GUARD({
        REQUIRE(ctx != nullptr && w != nullptr, "NULL argument");
        for (int l = 0; l < ctx->L; ++l) {
            REQUIRE(std::isfinite(w[l]), "weights must be finite");
            if (l >= 1) REQUIRE(w[l] >= 1.0, "Chebyshev alpha must be >= 1");
        }
        ctx->w.assign(w, w + ctx->L);
        write_cycle_tables(ctx);
        drop_graphs(ctx);
        ++ctx->data_gen;
        return HELM_OK;
    })
}

helm_status helm_get_weights(helm_ctx ctx, double* w) {
    ABI_GUARD({
        REQUIRE(ctx != nullptr && w != nullptr, "NULL argument");
        for (int l = 0; l < ctx->L; ++l) w[l] = ctx->w[l];
        return HELM_OK;
    })
}

helm_status helm_get_lambdas(helm_ctx ctx, double* lam) {
    ABI_GUARD({
        REQUIRE(ctx != nullptr && lam != nullptr, "NULL argument");
        for (int l = 1; l <= ctx->L; ++l) lam[l - 1] = ctx->wl[l].lam;
        return HELM_OK;
    })
}

helm_status helm_cycle(helm_ctx ctx, const void* g, void* u, void* stream) {
    ABI_GUARD({
        REQUIRE(ctx != nullptr && g != nullptr && u != nullptr, "NULL argument");
        if (ctx->d.adr_steps > 0 && ctx->L >= 3 && !ctx->phase_set)
            throw Error(HELM_ESTATE, "helm_set_phase must be called before helm_cycle");
        cycle_any(ctx, g, u, u, (hipStream_t)stream);
        HIPCHK(hipGetLastError());
        return HELM_OK;
    })
}

helm_status helm_solve(helm_ctx ctx, const void* g, void* u, double tol, int32_t maxit, int32_t mode,
                       int32_t* iters, double* relres, double* history, void* stream) {
    ABI_GUARD({
        REQUIRE(ctx != nullptr && g != nullptr && u != nullptr && iters != nullptr && relres != nullptr,
                "NULL argument");
        REQUIRE(tol > 0 && maxit >= 1, "tol must be > 0 and maxit >= 1");
        REQUIRE(mode == 0 || mode == 1, "mode must be 0 or 1");
        if (ctx->d.adr_steps > 0 && ctx->L >= 3 && !ctx->phase_set)
            throw Error(HELM_ESTATE, "helm_set_phase must be called before helm_solve");
        int it = 0;
        double rr = 0;
        helm_status s = solve(ctx, g, u, tol, maxit, mode, &it, &rr, history, (hipStream_t)stream);
        HIPCHK(hipGetLastError());
        *iters = it;
        *relres = rr;
        if (s == HELM_ENOCONV) g_last_error = "tolerance not reached within maxit";
        if (s == HELM_EBREAKDOWN) g_last_error = "breakdown: non-finite or growing residual";
        return s;
    })
}

helm_status helm_residual(helm_ctx ctx, const void* g, const void* u, void* r, double* rnorm, double* gnorm,
                          void* stream) {
    ABI_GUARD({
        REQUIRE(ctx != nullptr && g != nullptr && u != nullptr, "NULL argument");
        residual_fp64(ctx, (hipStream_t)stream, g, u, r, rnorm, gnorm);
        return HELM_OK;
    })
}

helm_status helm_residual_noalloc(helm_ctx ctx, const void* g, const void* u, void* r, double* rnorm,
                                  double* gnorm, void* stream) {
    ABI_GUARD({
        REQUIRE(ctx != nullptr && g != nullptr && u != nullptr, "NULL argument");
        residual_fp64_noalloc(ctx, (hipStream_t)stream, g, u, r, rnorm, gnorm);
        return HELM_OK;
    })
}

// Checks shared by the adjoint entry points.
static void adj_require(helm_ctx ctx, const char* who) {
    REQUIRE(ctx->nsets == 1, std::string(who) + " needs a single phase (helm_set_phase), not Wave-Ray phases");
    if (ctx->d.adr_steps > 0 && ctx->L >= 3 && !ctx->phase_set)
        throw Error(HELM_ESTATE, std::string("helm_set_phase must be called before ") + who);
    if (ctx->phase_factored)
        throw Error(HELM_ESTATE, std::string(who) + " needs a phase from helm_set_phase (the product-rule "
                                                    "coefficients of helm_eikonal have no adjoint)");
    REQUIRE(ctx->d.gmres_m <= GMAX && ctx->d.gmres_coarse_m <= GMAX, "the adjoint supports GMRES dimensions up to 6");
}

helm_status helm_cycle_backward(helm_ctx ctx, int32_t K, const void* g, const void* u0, const void* grad_uK,
                                void* grad_phi, double* grad_w, void* ckpt_ws, void* stream) {
    ABI_GUARD({
        REQUIRE(ctx != nullptr && g != nullptr && grad_uK != nullptr && grad_phi != nullptr && grad_w != nullptr,
                "NULL argument");
        REQUIRE(K >= 1 && K <= 100000, "K must be in [1, 100000]");
        adj_require(ctx, "helm_cycle_backward");
        hipStream_t st = (hipStream_t)stream;
        if (ctx->f32) cycle_backward<float>(ctx, K, g, u0, grad_uK, grad_phi, grad_w, ckpt_ws, st);
        else cycle_backward<double>(ctx, K, g, u0, grad_uK, grad_phi, grad_w, ckpt_ws, st);
        HIPCHK(hipGetLastError());
        return HELM_OK;
    })
}

helm_status helm_cycle_record(helm_ctx ctx, int32_t K, const void* g, const void* u0, void* u_out, void* ckpt_ws,
                              void* stream) {
    ABI_GUARD({
        REQUIRE(ctx != nullptr && g != nullptr && u_out != nullptr, "NULL argument");
        REQUIRE(K >= 1 && K <= 100000, "K must be in [1, 100000]");
        adj_require(ctx, "helm_cycle_record");
        hipStream_t st = (hipStream_t)stream;
        const bool ok = ctx->f32 ? cycle_record<float>(ctx, K, g, u0, u_out, ckpt_ws, st)
                                 : cycle_record<double>(ctx, K, g, u0, u_out, ckpt_ws, st);
        if (!ok)
            throw Error(HELM_ENOMEM, "helm_cycle_record: the K tapes do not fit (helm_cycle_backward records "
                                     "one cycle at a time)");
        HIPCHK(hipGetLastError());
        return HELM_OK;
    })
}

helm_status helm_cycle_reverse(helm_ctx ctx, int32_t K, const void* g, const void* grad_uK, void* grad_phi,
                               double* grad_w, void* stream) {
    ABI_GUARD({
        REQUIRE(ctx != nullptr && g != nullptr && grad_uK != nullptr && grad_phi != nullptr && grad_w != nullptr,
                "NULL argument");
        adj_require(ctx, "helm_cycle_reverse");
        const helm::AdjState* S = ctx->adj;
        if (!S || !S->rec_valid)
            throw Error(HELM_ESTATE, "helm_cycle_reverse needs the tapes of a helm_cycle_record (none, or "
                                     "rewritten by helm_cycle_backward)");
        if (S->rec_K != K || S->rec_g != g)
            throw Error(HELM_ESTATE, "helm_cycle_reverse: K and g must be those of the last helm_cycle_record");
        if (S->rec_gen != ctx->data_gen)
            throw Error(HELM_ESTATE, "helm_cycle_reverse: the phase or the weights changed since helm_cycle_record");
        hipStream_t st = (hipStream_t)stream;
        if (ctx->f32) cycle_reverse<float>(ctx, grad_uK, grad_phi, grad_w, st);
        else cycle_reverse<double>(ctx, grad_uK, grad_phi, grad_w, st);
        HIPCHK(hipGetLastError());
        return HELM_OK;
    })
}

helm_status helm_loss(helm_ctx ctx, const void* g, const void* u, double* loss, void* grad_u, void* stream) {
    ABI_GUARD({
        REQUIRE(ctx != nullptr && g != nullptr && u != nullptr && loss != nullptr, "NULL argument");
        hipStream_t st = (hipStream_t)stream;
        *loss = ctx->f32 ? loss_grad<float>(ctx, g, u, grad_u, st) : loss_grad<double>(ctx, g, u, grad_u, st);
        HIPCHK(hipGetLastError());
        return HELM_OK;
    })
}

helm_status helm_batch_setup(int32_t nprob, const helm_desc* desc, const double* const* velocity,
                             const void* const* phi, int32_t phi_is_f64, int32_t lanes, helm_batch* out,
                             void* stream) {
    ABI_GUARD({
        REQUIRE(out != nullptr && desc != nullptr && velocity != nullptr, "NULL argument");
        REQUIRE(nprob >= 1 && nprob <= 4096, "nprob must be in [1, 4096]");
        REQUIRE(lanes >= 0 && lanes <= 64, "lanes must be in [0, 64]");
        for (int p = 0; p < nprob; ++p) {
            validate(&desc[p]);
            REQUIRE(velocity[p] != nullptr, "velocity[" + std::to_string(p) + "] is NULL");
        }
        helm_batch b = new helm_batch_s();
        try {
            HIPCHK(hipGetDevice(&b->device));
            b->lanes = std::min(nprob, lanes > 0 ? lanes : 4);
            b->ctx.assign(nprob, nullptr);
            for (int l = 0; l < b->lanes; ++l) {
                hipStream_t s = nullptr;
                HIPCHK(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
                b->streams.push_back(s);
                hipEvent_t e = nullptr;
                HIPCHK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
                b->events.push_back(e);
            }
            HIPCHK(hipEventCreateWithFlags(&b->ev_in, hipEventDisableTiming));
            lanes_after(b, (hipStream_t)stream);
            // classes: equal descriptors in FP32 cycles, at most BMAX problems each; the others alone
            std::vector<int> single;
            std::vector<char> taken(nprob, 0);
            for (int p : longest_first_desc(desc, nprob)) {
                if (taken[p]) continue;
                taken[p] = 1;
                std::vector<int> members{p};
                if (desc[p].cycle_prec == HELM_C64)
                    for (int q = p + 1; q < nprob && (int)members.size() < BMAX; ++q)
                        if (!taken[q] && same_desc(desc[p], desc[q])) {
                            taken[q] = 1;
                            members.push_back(q);
                        }
                if (members.size() >= 2) {
                    helm_batch_s::Class K;
                    K.probs = members;
                    b->classes.push_back(K);
                } else {
                    single.push_back(p);
                }
            }
            for (auto& K : b->classes) {
                K.stride = class_stride(desc[K.probs[0]], velocity[K.probs[0]], b->streams[0]);
                HIPCHK(hipMalloc((void**)&K.arena, K.stride * K.probs.size()));
                const size_t gsz = sizeof(double) * (size_t)(MAXM + 1) * BMAX * CLASS_GATHER;
                HIPCHK(hipMalloc((void**)&K.dg, gsz));
                HIPCHK(hipHostMalloc((void**)&K.hg, gsz, hipHostMallocDefault));
                for (auto& e : K.ev) HIPCHK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
            }
            // build: every problem of a class in its region, the others on their own
            struct Item {
                int p, cls, q;
            };
            std::vector<Item> items;
            for (int k = 0; k < (int)b->classes.size(); ++k)
                for (int q = 0; q < (int)b->classes[k].probs.size(); ++q) items.push_back({b->classes[k].probs[q], k, q});
            for (int p : single) items.push_back({p, -1, 0});
            std::vector<helm_status> st(nprob, HELM_OK);
            std::vector<std::string> msg(nprob);
            run_jobs(b, (int)items.size(), [&](int j, int lane, bool dev_ok) {
                const Item it = items[j];
                try {
                    REQUIRE(dev_ok, "hipSetDevice failed on a lane thread");
                    const void* ph = phi ? phi[it.p] : nullptr;
                    if (it.cls >= 0) {
                        b->ctx[it.p] = class_build(b->classes[it.cls], it.q, desc[it.p], velocity[it.p], ph,
                                                   phi_is_f64 != 0, b->streams[lane]);
                    } else {
                        helm_ctx c = new helm_ctx_s();
                        c->d = desc_normalized(desc[it.p]);
                        b->ctx[it.p] = c;
                        build(c, velocity[it.p], b->streams[lane]);
                        if (ph) set_phase(c, ph, phi_is_f64 != 0, b->streams[lane]);
                    }
                } catch (const Error& e) {
                    st[it.p] = e.code;
                    msg[it.p] = e.what();
                } catch (const std::exception& e) {
                    st[it.p] = HELM_EHIP;
                    msg[it.p] = e.what();
                }
            });
            helm_status s = first_error(st, msg);
            if (s != HELM_OK) throw Error(s, g_last_error);
            caller_after(b, (hipStream_t)stream);
        } catch (...) {
            batch_free(b);
            throw;
        }
        *out = b;
        return HELM_OK;
    })
}

helm_status helm_batch_get(helm_batch b, int32_t p, helm_ctx* out) {
    ABI_GUARD({
        REQUIRE(b != nullptr && out != nullptr, "NULL argument");
        REQUIRE(p >= 0 && p < (int)b->ctx.size(), "problem index out of range");
        *out = b->ctx[p];
        return HELM_OK;
    })
}

helm_status helm_batch_solve(helm_batch b, const void* const* g, void* const* u, double tol, int32_t maxit,
                             int32_t mode, int32_t* iters, double* relres, int32_t* status, void* stream) {
    ABI_GUARD({
        REQUIRE(b != nullptr && g != nullptr && u != nullptr && iters != nullptr && relres != nullptr &&
                    status != nullptr,
                "NULL argument");
        REQUIRE(tol > 0 && maxit >= 1, "tol must be > 0 and maxit >= 1");
        REQUIRE(mode == 0 || mode == 1, "mode must be 0 or 1");
        const int np = (int)b->ctx.size();
        for (int p = 0; p < np; ++p) {
            REQUIRE(g[p] != nullptr && u[p] != nullptr, "g[p] and u[p] must not be NULL");
            helm_ctx c = b->ctx[p];
            if (c->d.adr_steps > 0 && c->L >= 3 && !c->phase_set)
                throw Error(HELM_ESTATE, "problem " + std::to_string(p) + ": phase not set");
            if (mode == 1) REQUIRE(c->f32, "mode 1 needs cycle_prec = HELM_C64 for every problem");
        }
        lanes_after(b, (hipStream_t)stream);
        // jobs: the classes that can run in lockstep (mode 1), then every other problem alone,
        // the largest amount of work first
        struct Job {
            int cls, p;
            double work;
        };
        std::vector<Job> jobs;
        std::vector<char> in_class(np, 0);
        if (mode == 1)
            for (int k = 0; k < (int)b->classes.size(); ++k)
                if (class_lockstep_ok(b, b->classes[k])) {
                    const auto& K = b->classes[k];
                    for (int p : K.probs) in_class[p] = 1;
                    jobs.push_back({k, -1, NN2(b->ctx[K.probs[0]]->d.n, b->ctx[K.probs[0]]->d.ny) * K.probs.size()});
                }
        for (int p = 0; p < np; ++p)
            if (!in_class[p]) jobs.push_back({-1, p, NN2(b->ctx[p]->d.n, b->ctx[p]->d.ny)});
        std::stable_sort(jobs.begin(), jobs.end(), [](const Job& a, const Job& c) { return a.work > c.work; });
        b->last_class.assign(np, -1);
        for (const Job& jb : jobs)
            if (jb.cls >= 0)
                for (int p : b->classes[jb.cls].probs) b->last_class[p] = jb.cls;
        std::vector<helm_status> st(np, HELM_OK);
        std::vector<std::string> msg(np);
        run_jobs(b, (int)jobs.size(), [&](int j, int lane, bool dev_ok) {
            const Job jb = jobs[j];
            auto fail_all = [&](helm_status code, const std::string& m) {
                if (jb.cls >= 0) {
                    for (int p : b->classes[jb.cls].probs) {
                        st[p] = code;
                        msg[p] = m;
                    }
                } else {
                    st[jb.p] = code;
                    msg[jb.p] = m;
                }
            };
            try {
                REQUIRE(dev_ok, "hipSetDevice failed on a lane thread");
                if (jb.cls >= 0) {
                    class_solve(b, b->classes[jb.cls], g, u, tol, maxit, iters, relres, st, b->streams[lane]);
                } else {
                    int it = 0;
                    double rr = 0.0;
                    st[jb.p] = solve(b->ctx[jb.p], g[jb.p], u[jb.p], tol, maxit, mode, &it, &rr, nullptr,
                                     b->streams[lane]);
                    HIPCHK(hipGetLastError());
                    iters[jb.p] = it;
                    relres[jb.p] = rr;
                }
            } catch (const Error& e) {
                fail_all(e.code, e.what());
            } catch (const std::exception& e) {
                fail_all(HELM_EHIP, e.what());
            }
            if (jb.cls >= 0) b->ctx[b->classes[jb.cls].probs[0]]->bi = BatchIdx{};
        });
        for (int p = 0; p < np; ++p) status[p] = st[p];
        caller_after(b, (hipStream_t)stream);
        return first_error(st, msg);
    })
}

helm_status helm_batch_classes(helm_batch b, int32_t* class_of) {
    ABI_GUARD({
        REQUIRE(b != nullptr && class_of != nullptr, "NULL argument");
        for (size_t p = 0; p < b->ctx.size(); ++p)
            class_of[p] = p < b->last_class.size() ? b->last_class[p] : -1;
        return HELM_OK;
    })
}

helm_status helm_batch_destroy(helm_batch b) {
    batch_free(b);
    return HELM_OK;
}

helm_status helm_tune(helm_ctx ctx, char* json, int64_t cap, void* stream) {
    ABI_GUARD({
        REQUIRE(ctx != nullptr, "NULL argument");
        hipStream_t st = (hipStream_t)stream;
        std::string out = ctx->f32 ? tune_ctx<float>(ctx, st) : tune_ctx<double>(ctx, st);
        if (json) {
            REQUIRE((int64_t)out.size() < cap, "tuning buffer too small");
            std::memcpy(json, out.c_str(), out.size() + 1);
        }
        return HELM_OK;
    })
}

helm_status helm_set_tuning(helm_ctx ctx, const char* json) {
    ABI_GUARD({
        REQUIRE(ctx != nullptr && json != nullptr, "NULL argument");
        apply_tuning(ctx, json);
        return HELM_OK;
    })
}

helm_status helm_get_tuning(helm_ctx ctx, char* json, int64_t cap) {
    ABI_GUARD({
        REQUIRE(ctx != nullptr && json != nullptr && cap > 0, "NULL argument");
        std::string out = tuning_json(ctx, "");
        REQUIRE((int64_t)out.size() < cap, "tuning buffer too small");
        std::memcpy(json, out.c_str(), out.size() + 1);
        return HELM_OK;
    })
}

helm_status helm_debug_op(helm_ctx ctx, int32_t op, int32_t level, const void* in, const void* in2, void* out,
                          void* stream) {
    ABI_GUARD({
        REQUIRE(ctx != nullptr && out != nullptr, "NULL argument");
        REQUIRE(level >= 1 && level <= ctx->L, "bad level");
        hipStream_t st = (hipStream_t)stream;
        auto run = [&](auto tag) {
            using T = decltype(tag);
            Engine<T> E(ctx, st);
            WaveLevel& W = ctx->wl[level];
            switch (op) {
                case 1:
                    if (W.f64) E.template applyA<double>(W.G, W.n2, in, out, 0);
                    else E.template applyA<T>(W.G, W.n2, in, out, 0);
                    break;
                case 2:
                    REQUIRE(level < ctx->L, "restriction needs level < L");
                    if (ctx->wl[level + 1].f64 && !W.f64) {
                        // in -> R in with g = in, u = 0
                        E.template resid_restrict<T, double>(level, in, nullptr, out);
                    } else if (W.f64) {
                        E.template resid_restrict<double, double>(level, in, nullptr, out);
                    } else {
                        E.template resid_restrict<T, T>(level, in, nullptr, out);
                    }
                    break;
                case 3:
                    REQUIRE(level < ctx->L, "prolongation needs level < L");
                    if (ctx->wl[level + 1].f64 && !W.f64) E.template prolong_add<double, T>(level, in, out);
                    else if (W.f64) E.template prolong_add<double, double>(level, in, out);
                    else E.template prolong_add<T, T>(level, in, out);
                    break;
                case 4:
                    REQUIRE(level == 1, "Jacobi runs on level 1");
                    hipLaunchKernelGGL((k_jacobi<T>), dim3(tiles_of(W.nx, W.ny)), tile_block(), 0, st, W.G, (const T*)W.n2,
                                       (const cplx<T>*)in2, (const cplx<T>*)in, (cplx<T>*)out,
                                       (const double*)ctx->cdev->la, BatchIdx{});
                    break;
                case 5: {
                    REQUIRE(level >= 2, "Chebyshev runs on levels >= 2");
                    const size_t Nl = (size_t)W.nx * W.ny;
                    const int m = (level == ctx->L) ? ctx->d.cheb_coarse : ctx->d.cheb_pre;
                    if (W.f64) {
                        HIPCHK(hipMemcpyAsync(out, in, Nl * sizeof(c128), hipMemcpyDeviceToDevice, st));
                        E.template chebyshev<double>(level, in2, out, false, ctx->w[level - 1], m);
                    } else {
                        HIPCHK(hipMemcpyAsync(out, in, Nl * sizeof(cplx<T>), hipMemcpyDeviceToDevice, st));
                        E.template chebyshev<T>(level, in2, out, false, ctx->w[level - 1], m);
                    }
                    break;
                }
                case 6: {
                    REQUIRE(level >= 2 && level <= ctx->LA && ctx->L >= 3 && ctx->phase_set,
                            "ADR operator needs the phase and an ADR level");
                    AdrLevel& A = ctx->al[level];
                    hipLaunchKernelGGL((k_adr_apply<T>), dim3(tiles_of(A.nx, A.ny)), tile_block(), 0, st, A.A,
                                       (const T*)A.px, (const T*)A.py, (const cplx<T>*)A.c0, (const cplx<T>*)in,
                                       (cplx<T>*)out, BatchIdx{});
                    break;
                }
                case 7: {
                    REQUIRE(level >= 2 && ctx->L >= 3 && ctx->phase_set, "GMRES needs the phase");
                    AdrLevel& A = ctx->al[level];
                    const size_t Nl = (size_t)A.nx * A.ny;
                    HIPCHK(hipMemcpyAsync(A.b, in2, Nl * sizeof(cplx<T>), hipMemcpyDeviceToDevice, st));
                    HIPCHK(hipMemcpyAsync(A.x, in, Nl * sizeof(cplx<T>), hipMemcpyDeviceToDevice, st));
                    REQUIRE(level <= ctx->LA, "level beyond the ADR hierarchy");
                    E.gmres(level, level == ctx->LA ? ctx->d.gmres_coarse_m : ctx->d.gmres_m, false);
                    HIPCHK(hipMemcpyAsync(out, A.x, Nl * sizeof(cplx<T>), hipMemcpyDeviceToDevice, st));
                    break;
                }
                case 8: {
                    REQUIRE(level >= 2 && ctx->L >= 3 && ctx->phase_set, "ADR V-cycle needs the phase");
                    AdrLevel& A = ctx->al[level];
                    const size_t Nl = (size_t)A.nx * A.ny;
                    HIPCHK(hipMemcpyAsync(A.b, in2, Nl * sizeof(cplx<T>), hipMemcpyDeviceToDevice, st));
                    E.adr_vcycle(level);
                    HIPCHK(hipMemcpyAsync(out, A.x, Nl * sizeof(cplx<T>), hipMemcpyDeviceToDevice, st));
                    break;
                }
                case 9: {
                    REQUIRE(level == 2 && ctx->L >= 3 && ctx->phase_set, "ADR step runs on level 2 with the phase");
                    const size_t Nl = (size_t)W.nx * W.ny;
                    HIPCHK(hipMemcpyAsync(W.g, in2, Nl * sizeof(cplx<T>), hipMemcpyDeviceToDevice, st));
                    HIPCHK(hipMemcpyAsync(W.u, in, Nl * sizeof(cplx<T>), hipMemcpyDeviceToDevice, st));
                    E.adr_steps(1);
                    HIPCHK(hipMemcpyAsync(out, W.u, Nl * sizeof(cplx<T>), hipMemcpyDeviceToDevice, st));
                    break;
                }
                case 10: {
                    if (level == 1) {
                        E.cycle(in2, in, out);
                    } else {
                        REQUIRE(in == nullptr, "coarse cycles start from a zero iterate (in must be NULL)");
                        const size_t Nl = (size_t)W.nx * W.ny;
                        HIPCHK(hipMemcpyAsync(W.g, in2, Nl * csize(W.f64), hipMemcpyDeviceToDevice, st));
                        E.cycle_coarse(level);
                        HIPCHK(hipMemcpyAsync(out, W.u, Nl * csize(W.f64), hipMemcpyDeviceToDevice, st));
                    }
                    break;
                }
                case 11:
                    REQUIRE(level < ctx->L, "restriction needs level < L");
                    if (W.f64) E.template resid_restrict<double, double>(level, in2, in, out);
                    else if (ctx->wl[level + 1].f64) E.template resid_restrict<T, double>(level, in2, in, out);
                    else E.template resid_restrict<T, T>(level, in2, in, out);
                    break;
                case 12: {
                    // plain copy of one level's complex array (a known-size probe for
                    // hardware memory counters)
                    const size_t Nl = (size_t)W.nx * W.ny;
                    if (W.f64)
                        LAUNCH(ctx, 32.0 * Nl, (k_copy<double>), dim3(flat_blocks(Nl, 8192)), dim3(BLOCK), st, Nl,
                               (const c128*)in, (c128*)out);
                    else
                        LAUNCH(ctx, 2.0 * sizeof(cplx<T>) * Nl, (k_copy<T>), dim3(flat_blocks(Nl, 8192)), dim3(BLOCK),
                               st, Nl, (const cplx<T>*)in, (cplx<T>*)out);
                    break;
                }
                default:
                    throw Error(HELM_EINVAL, "unknown debug op");
            }
        };
        if (ctx->f32) run(float{});
        else run(double{});
        HIPCHK(hipGetLastError());
        HIPCHK(hipStreamSynchronize(st));
        return HELM_OK;
    })
}

helm_status helm_profile_begin(helm_ctx ctx) {
    ABI_GUARD({
        REQUIRE(ctx != nullptr, "NULL argument");
        ctx->prof.recs.clear();
        ctx->prof.used = 0;
        ctx->prof.on = true;
        return HELM_OK;
    })
}

helm_status helm_profile_end(helm_ctx ctx, char* json, int64_t cap) {
    ABI_GUARD({
        REQUIRE(ctx != nullptr && json != nullptr && cap > 0, "NULL argument");
        auto& P = ctx->prof;
        P.on = false;
        if (!P.recs.empty()) HIPCHK(hipEventSynchronize(P.recs.back().e1));
        // Launches are grouped by kernel and grid; a group whose launches move one of at
        // most three distinct byte counts (the same kernel on different levels with the
        // same grid) is split by byte count, one whose byte count varies from launch to
        // launch (a Krylov pass over a growing basis) stays whole.
        struct Agg {
            std::string name;
            long launches = 0;
            double ms = 0, bytes = 0;
        };
        struct Sub {
            std::string base;
            double bpl;
            long launches = 0;
            double ms = 0, bytes = 0;
        };
        std::vector<Sub> subs;
        for (auto& r : P.recs) {
            float ms = 0.f;
            HIPCHK(hipEventElapsedTime(&ms, r.e0, r.e1));
            std::string base = std::string(r.name) + " [" + std::to_string(r.grid) + " blocks";
            auto it = std::find_if(subs.begin(), subs.end(),
                                   [&](const Sub& a) { return a.base == base && a.bpl == r.bytes; });
            if (it == subs.end()) {
                subs.push_back(Sub{base, r.bytes});
                it = subs.end() - 1;
            }
            it->launches += 1;
            it->ms += ms;
            it->bytes += r.bytes;
        }
        std::vector<Agg> agg;
        for (auto& sb : subs) {
            const long distinct = std::count_if(subs.begin(), subs.end(), [&](const Sub& a) { return a.base == sb.base; });
            std::string key = sb.base + "]";
            if (distinct <= 3) {
                char mb[48];
                std::snprintf(mb, sizeof(mb), ", %.1f MB", sb.bpl / 1e6);
                key = sb.base + mb + "]";
            }
            auto it = std::find_if(agg.begin(), agg.end(), [&](const Agg& a) { return a.name == key; });
            if (it == agg.end()) {
                agg.push_back(Agg{key});
                it = agg.end() - 1;
            }
            it->launches += sb.launches;
            it->ms += sb.ms;
            it->bytes += sb.bytes;
        }
        std::sort(agg.begin(), agg.end(), [](const Agg& a, const Agg& b) { return a.ms > b.ms; });
        std::string out = "{\"kernels\": [";
        for (size_t i = 0; i < agg.size(); ++i) {
            char buf[512];
            std::string nm = agg[i].name;
            for (auto& ch : nm)
                if (ch == '"') ch = '\'';
            std::snprintf(buf, sizeof(buf), "%s{\"name\": \"%s\", \"launches\": %ld, \"ms\": %.6f, \"bytes\": %.6e}",
                          i ? ", " : "", nm.c_str(), agg[i].launches, agg[i].ms, agg[i].bytes);
            out += buf;
        }
        out += "]}";
        P.recs.clear();
        P.used = 0;
        REQUIRE((int64_t)out.size() < cap, "profile buffer too small");
        std::memcpy(json, out.c_str(), out.size() + 1);
        return HELM_OK;
    })
}

helm_status helm_destroy(helm_ctx ctx) {
    if (!ctx) return HELM_OK;
    drop_graphs(ctx);
    delete ctx->adj;
    ctx->adj = nullptr;
    if (ctx->cap_stream) (void)hipStreamDestroy(ctx->cap_stream);
    for (hipEvent_t e : ctx->prof.pool) (void)hipEventDestroy(e);
    for (hipEvent_t e : ctx->col_ev)
        if (e) (void)hipEventDestroy(e);
    if (ctx->hcol) (void)hipHostFree(ctx->hcol);
    ctx->prof.pool.clear();
    for (void* p : ctx->allocs) (void)hipFree(p);
    ctx->allocs.clear();
    delete ctx;
    return HELM_OK;
}

const char* helm_status_string(helm_status s) {
    switch (s) {
        case HELM_OK: return "HELM_OK";
        case HELM_EINVAL: return "HELM_EINVAL: invalid argument";
        case HELM_ENOMEM: return "HELM_ENOMEM: device allocation failed";
        case HELM_EHIP: return "HELM_EHIP: HIP runtime error";
        case HELM_ENOCONV: return "HELM_ENOCONV: tolerance not reached";
        case HELM_EBREAKDOWN: return "HELM_EBREAKDOWN: numerical breakdown";
        case HELM_ESTATE: return "HELM_ESTATE: call out of order";
    }
    return "unknown status";
}

const char* helm_last_error(void) { return g_last_error.c_str(); }

const char* helm_version(void) { return "helm-mi355x 0.1 (gfx950)"; }

}  // extern "C"
