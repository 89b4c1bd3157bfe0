// Host side of the adjoint of K unrolled cycles (Section 3.3: the loss after K
// cycles and its back-propagation to the phase and to the smoother weights).
//
// Strategy: the K cycles are run forward from u_0 while a tape per cycle records what
// its reverse needs (the inputs of the smoothers, the ADR right-hand sides and
// iterates, and for every GMRES call the monomial Krylov basis and its least-squares
// record); u_{k+1} comes from that recording.  Then, for k = K-1 .. 0, cycle k is
// reversed from its tape: u_k's cotangent from u_{k+1}'s, with the cotangents of the
// weights, of the ADR coefficients phi_x, phi_y, c0 and of the carrier phase
// accumulated on the way.  At the end those are pulled back to the fine phase.  When K
// tapes do not fit, one tape is reused: the K forward cycles are run first for the
// checkpoints u_k, and each cycle is recorded again from u_k just before its reverse.
//
// Included from helm.hip inside namespace helm (uses its context, LAUNCH, Engine).
#pragma once

struct AdrTape {  // one GMRES-smoothed ADR level inside one ADR step
    void* b = nullptr;
    void* x1 = nullptr;
    void* x2 = nullptr;
    void* xo = nullptr;
    void* kpre[GMAX + 1] = {};
    void* kpost[GMAX + 1] = {};
    GRec* rpre = nullptr;
    GRec* rpost = nullptr;
};

// What the reverse of one cycle reads: the tape of its recording.
struct CycleTape {
    void* uB = nullptr;                      // level 1: input of the post-Jacobi sweep
    std::vector<void*> g, ub;                // wave levels: right-hand side, input of the post-smoother
    std::vector<std::vector<AdrTape>> adr;   // [step][level]
};

struct AdjState {
    bool ready = false;
    int M = 0;
    size_t tape_bytes = 0;                   // device bytes of one cycle's tape
    std::vector<CycleTape> tapes;            // one per cycle when they fit, else one reused per cycle
    int cur = 0;                             // the tape being recorded or reversed
    void* ubuf = nullptr;                    // u_k of the cycle being reversed (graph input, one tape)
    void* fb[2] = {};                        // level-1 cotangents
    std::vector<void*> lub, lgb;             // cotangent of the level's output / of its right-hand side
    std::vector<std::array<void*, 9>> cs;    // Chebyshev reverse scratch
    std::vector<void*> axb, axb2, abb, acc0, acc1;  // ADR cotangents per level
    std::vector<double*> pxb, pyb;
    std::vector<c128*> c0b;
    double* thb = nullptr;                   // carrier phase cotangent (level 2)
    double* phib2 = nullptr;                 // phase cotangent on the level-2 lattice
    double* wacc = nullptr;                  // weight cotangents (FP64, device)
    double* wpart = nullptr;                 // WSLOTS x MAXRED partials of weight cotangents
    void* ckpt = nullptr;                    // library-owned checkpoints
    size_t ckpt_bytes = 0;
    // the tapes of helm_cycle_record, reversible by helm_cycle_reverse while valid
    void* uK = nullptr;                      // u_K of the recording (graph output, copied out)
    bool rec_valid = false;
    int rec_K = 0;
    const void* rec_g = nullptr;
    char* rec_ck = nullptr;
    uint64_t rec_gen = 0;
};

static void dfree(helm_ctx c, void* p) {
    if (!p) return;
    auto it = std::find(c->allocs.begin(), c->allocs.end(), p);
    if (it != c->allocs.end()) c->allocs.erase(it);
    (void)hipFree(p);
}

static int gm_of(helm_ctx c, int l) { return l == c->LA ? c->d.gmres_coarse_m : c->d.gmres_m; }

// One cycle's tape: the wave-level inputs, and per ADR step and level the right-hand
// side, iterates, Krylov bases (zeroed here: the tile record leaves their ring unwritten)
// and GMRES records.
static void alloc_tape(helm_ctx c, CycleTape& T, int M, hipStream_t st) {
    const int L = c->L;
    const bool f64c = !c->f32;
    const size_t NF = (size_t)c->d.n * c->d.ny;
    T.uB = dalloc(c, NF * csize(f64c));
    T.g.assign(L + 1, nullptr);
    T.ub.assign(L + 1, nullptr);
    for (int l = 2; l <= L; ++l) {
        const size_t cb = (size_t)lnx(c, l) * lny(c, l) * csize(c->wl[l].f64);
        T.g[l] = dalloc(c, cb);
        if (l < L) T.ub[l] = dalloc(c, cb);
    }
    if (M == 0) return;
    T.adr.assign(M, std::vector<AdrTape>(c->LA + 1));
    const int nrec = M * c->LA * 2;
    GRec* recs = (GRec*)dalloc(c, (size_t)nrec * sizeof(GRec));
    std::vector<GRec> hrec(nrec);
    std::memset(hrec.data(), 0, hrec.size() * sizeof(GRec));
    int ri = 0;
    for (int l = 2; l <= c->LA; ++l) {
        const size_t cb = (size_t)lnx(c, l) * lny(c, l) * csize(f64c);
        const int m = gm_of(c, l);
        for (int s = 0; s < M; ++s) {
            AdrTape& A = T.adr[s][l];
            A.b = dalloc(c, cb);
            A.xo = dalloc(c, cb);
            for (int q = 0; q <= m; ++q) {
                A.kpre[q] = dalloc(c, cb);
                HIPCHK(hipMemsetAsync(A.kpre[q], 0, cb, st));
            }
            hrec[ri].m = m;
            A.rpre = recs + ri++;
            if (l < c->LA) {
                A.x1 = dalloc(c, cb);
                A.x2 = dalloc(c, cb);
                for (int q = 0; q <= m; ++q) {
                    A.kpost[q] = dalloc(c, cb);
                    HIPCHK(hipMemsetAsync(A.kpost[q], 0, cb, st));
                }
                hrec[ri].m = m;
                A.rpost = recs + ri++;
            }
        }
    }
    HIPCHK(hipMemcpyAsync(recs, hrec.data(), hrec.size() * sizeof(GRec), hipMemcpyHostToDevice, st));
    HIPCHK(hipStreamSynchronize(st));
}

static void adj_alloc(helm_ctx c, hipStream_t st) {
    AdjState& S = *c->adj;
    if (S.ready) return;
    const int L = c->L;
    const bool f64c = !c->f32;
    const size_t NF = (size_t)c->d.n * c->d.ny;
    const bool adr_on = c->d.adr_steps > 0 && L >= 3;
    S.M = adr_on ? c->d.adr_steps : 0;
    S.ubuf = dalloc(c, NF * csize(f64c));
    S.fb[0] = dalloc(c, NF * csize(f64c));
    S.fb[1] = dalloc(c, NF * csize(f64c));
    S.lub.assign(L + 1, nullptr);
    S.lgb.assign(L + 1, nullptr);
    S.cs.assign(L + 1, {});
    for (int l = 2; l <= L; ++l) {
        const size_t cb = (size_t)lnx(c, l) * lny(c, l) * csize(c->wl[l].f64);
        S.lub[l] = dalloc(c, cb);
        S.lgb[l] = dalloc(c, cb);
        for (int q = 0; q < 9; ++q) S.cs[l][q] = dalloc(c, cb);
    }
    S.wacc = (double*)dalloc(c, 64 * sizeof(double));
    S.wpart = (double*)dalloc(c, (size_t)WSLOTS * MAXRED * sizeof(double));
    if (adr_on) {
        S.axb.assign(c->LA + 1, nullptr);
        S.axb2.assign(c->LA + 1, nullptr);
        S.abb.assign(c->LA + 1, nullptr);
        S.acc0.assign(c->LA + 1, nullptr);
        S.acc1.assign(c->LA + 1, nullptr);
        S.pxb.assign(c->LA + 1, nullptr);
        S.pyb.assign(c->LA + 1, nullptr);
        S.c0b.assign(c->LA + 1, nullptr);
        for (int l = 2; l <= c->LA; ++l) {
            const size_t Nl = (size_t)lnx(c, l) * lny(c, l);
            const size_t cb = Nl * csize(f64c);
            S.axb[l] = dalloc(c, cb);
            S.axb2[l] = dalloc(c, cb);
            S.abb[l] = dalloc(c, cb);
            S.acc0[l] = dalloc(c, cb);
            S.acc1[l] = dalloc(c, cb);
            // the tile reverse writes the unknowns only: rings stay at this 0
            for (void* z : {S.axb[l], S.axb2[l], S.abb[l], S.acc0[l], S.acc1[l]}) HIPCHK(hipMemsetAsync(z, 0, cb, st));
            S.pxb[l] = (double*)dalloc(c, Nl * sizeof(double));
            S.pyb[l] = (double*)dalloc(c, Nl * sizeof(double));
            S.c0b[l] = (c128*)dalloc(c, Nl * sizeof(c128));
        }
        const size_t N2 = (size_t)lnx(c, 2) * lny(c, 2);
        S.thb = (double*)dalloc(c, N2 * sizeof(double));
        S.phib2 = (double*)dalloc(c, N2 * sizeof(double));
    }
    const size_t before = c->count_bytes;
    S.tapes.assign(1, CycleTape{});
    alloc_tape(c, S.tapes[0], S.M, st);
    S.tape_bytes = c->count_bytes - before;
    HIPCHK(hipStreamSynchronize(st));
    S.ready = true;
}

// One tape per cycle when K of them fit (at most a quarter of the free device memory and
// 32 GiB, or HELM_ADJ_TAPE_MB MiB when that variable is set): the forward pass then
// records every cycle once and the checkpoint pass is not needed.  Returns whether K
// tapes are available.
static bool adj_tapes_for(helm_ctx c, int K, hipStream_t st) {
    AdjState& S = *c->adj;
    if ((int)S.tapes.size() >= K) return true;
    size_t fr = 0, tot = 0;
    HIPCHK(hipMemGetInfo(&fr, &tot));
    size_t cap = (size_t)32 << 30;
    if (const char* e = std::getenv("HELM_ADJ_TAPE_MB")) cap = (size_t)std::strtoull(e, nullptr, 10) << 20;
    const size_t need = (size_t)(K - (int)S.tapes.size()) * S.tape_bytes;
    if (need > fr / 4 || need > cap) return false;
    while ((int)S.tapes.size() < K) {
        S.tapes.emplace_back();
        alloc_tape(c, S.tapes.back(), S.M, st);
    }
    return true;
}

template <typename T>
struct AdjEngine {
    helm_ctx c;
    hipStream_t st;
    Engine<T> E;
    AdjState& S;
    using C = cplx<T>;

    AdjEngine(helm_ctx ctx, hipStream_t s) : c(ctx), st(s), E(ctx, s), S(*ctx->adj) {}

    CycleTape& tp() { return S.tapes[S.cur]; }

    size_t N(int l) const { return E.N(l); }
    int fb(size_t n) const { return flat_blocks(n); }
    double tau(int l) const { return 8.0 * c->al[l].A.inv_h2; }

    template <typename F>
    void prec(int l, F&& f) {
        if (c->wl[l].f64) f(double{});
        else f(T{});
    }
    void copy(void* dst, const void* src, size_t bytes) {
        HIPCHK(hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToDevice, st));
    }
    // Weight-cotangent partials: the passes that form them write to the next slot of S.wpart
    // (wslot()); fin_add(nblk, level) queues that slot, and wflush() sums the queued slots
    // into wacc in one launch (when WSLOTS are queued, and at the end of every reversed cycle).
    WSlots wq{};
    double* wslot() { return S.wpart + (size_t)wq.n * MAXRED; }
    void fin_add(int nblk, int level) {
        wq.nblk[wq.n] = nblk;
        wq.level[wq.n] = level;
        if (++wq.n == WSLOTS) wflush();
    }
    void wflush() {
        if (wq.n == 0) return;
        LAUNCH_NB(c, 8.0 * MAXRED * wq.n, k_wsum, dim3(1), dim3(FBLOCK), st, (const double*)S.wpart, MAXRED, wq,
                  S.wacc);
        wq = WSlots{};
    }

    // ------------------------------------------------------------ record (forward with tape)
    void rec_cycle(const void* g, const void* u0) {
        WaveLevel& W = c->wl[1];
        const Geom& G = W.G;
        LAUNCH(c, ((u0 ? 3 : 2) * sizeof(C) + sizeof(T)) * NN2(G.nx, G.ny), (k_jacobi<T>), dim3(tiles_of(G.nx, G.ny)), tile_block(),
               st, G, (const T*)W.n2, (const C*)g, (const C*)u0, (C*)tp().uB, (const double*)c->cdev->la);
        E.restrict_down(1, g, tp().uB, tp().g[2]);
        rec_level(2);
        E.prolong_up(1, c->wl[2].u, tp().uB);
    }

    // u_{k+1} = the post-Jacobi sweep of the recorded cycle (from the tape's uB).
    void post_jacobi(const void* g, void* out) {
        WaveLevel& W = c->wl[1];
        const Geom& G = W.G;
        LAUNCH(c, (3 * sizeof(C) + sizeof(T)) * NN2(G.nx, G.ny), (k_jacobi<T>), dim3(tiles_of(G.nx, G.ny)),
               tile_block(), st, G, (const T*)W.n2, (const C*)g, (const C*)tp().uB, (C*)out,
               (const double*)c->cdev->la);
    }

    void rec_level(int l) {
        WaveLevel& W = c->wl[l];
        const int L = c->L;
        const size_t cb = N(l) * csize(W.f64);
        if (l == L) {
            E.template chebyshev<double>(l, tp().g[l], W.u, true, c->w[l - 1], c->d.cheb_coarse);
            return;
        }
        if (l == 3) {
            E.restrict_down(l, tp().g[l], nullptr, tp().g[l + 1]);
        } else {
            E.template chebyshev<T>(l, tp().g[l], W.u, true, c->w[l - 1], c->d.cheb_pre);
            E.restrict_down(l, tp().g[l], W.u, tp().g[l + 1]);
        }
        rec_level(l + 1);
        if (l == 3) E.template zero<T>(W.u, N(l));
        E.prolong_up(l, c->wl[l + 1].u, W.u);
        if (l != 3 || c->d.level3_literal) {
            copy(tp().ub[l], W.u, cb);
            E.template chebyshev<T>(l, tp().g[l], W.u, false, c->w[l - 1], c->d.cheb_post);
        }
        if (l == 2)
            if (S.M > 0) rec_adr_steps();
    }

    // The ADR steps of level 2: the first demodulation, then per step the ADR V-cycle and
    // the re-modulation fused with the next step's demodulation; the iterate alternates
    // between W.u and W.ualt and ends in W.u.
    void rec_adr_steps() {
        WaveLevel& W = c->wl[2];
        const int M = S.M;
        LAUNCH(c, (4 * sizeof(C) + sizeof(T)) * NN2(W.nx, W.ny), (k_adr_demod<T>), dim3(tiles_of(W.nx, W.ny)),
               tile_block(), st, W.G, (const T*)W.n2, (const C*)tp().g[2], (const C*)W.u, (const C*)c->car2,
               (C*)tp().adr[0][2].b);
        void* ucur = W.u;
        void* unext = W.ualt;
        for (int s = 0; s < M; ++s) {
            rec_adrv(s, 2);
            const bool last = s + 1 == M;
            void* out = last ? W.u : unext;  // the last step lands in W.u (in place when it is current)
            if (last && ucur == W.u) {
                LAUNCH(c, 4 * sizeof(C) * double(N(2)), (k_adr_modadd<T>), dim3(fb(N(2))), dim3(BLOCK), st, N(2),
                       (const C*)tp().adr[s][2].xo, (const C*)c->car2, (C*)W.u);
                break;
            }
            LAUNCH_NB(c, (last ? 4.0 : 7.0) * sizeof(C) * double(N(2)), (k_adr_modadd_demod<T>), dim3(fb(N(2))),
                      dim3(BLOCK), st, W.G, (const T*)W.n2, (const C*)tp().g[2], (const C*)ucur,
                      (const C*)tp().adr[s][2].xo, (const C*)c->car2, (C*)out,
                      (C*)(last ? nullptr : tp().adr[s + 1][2].b));
            std::swap(ucur, unext);
        }
    }

    // pa_base, pa_out (level l - 1, may be null): the last call's result also goes to
    // pa_out = pa_base + P x (the finer level's post-smoother start).
    void rec_adrv(int s, int l, const void* pa_base = nullptr, void* pa_out = nullptr) {
        AdrTape& Tp = tp().adr[s][l];
        if (l == c->LA) {
            rec_gmres(l, Tp.b, nullptr, gm_of(c, l), Tp.kpre, Tp.rpre, Tp.xo, nullptr, pa_base, pa_out);
            return;
        }
        const int m = gm_of(c, l);
        rec_gmres(l, Tp.b, nullptr, m, Tp.kpre, Tp.rpre, Tp.x1, tp().adr[s][l + 1].b);
        rec_adrv(s, l + 1, Tp.x1, Tp.x2);
        rec_gmres(l, Tp.b, Tp.x2, m, Tp.kpost, Tp.rpost, Tp.xo, nullptr, pa_base, pa_out);
    }

    // The basis and Gram partials of a recorded GMRES(MM) call in one tile pass; returns
    // the number of blocks (whose partials k_gr_solve sums).
    template <int MM>
    int rec_tile(int l, const void* b, const void* x0, void* const* kv) {
        AdrLevel& A = c->al[l];
        KvOut<T> ko{};
        for (int q = 0; q <= MM; ++q) ko.v[q] = (C*)kv[q];
        const int tt = E.sstep_tile_edge(l) == 16 ? 16 : 32;
        int nb = 0;
        const double bytes = ((x0 ? 3.0 : 2.0) * sizeof(C) + 2 * sizeof(T)) * double(N(l)) +
                             (MM + 1.0) * sizeof(C) * double(N(l));
        auto go = [&](auto ttc, auto x0c) {
            constexpr int TT = decltype(ttc)::value;
            constexpr bool X0 = decltype(x0c)::value;
            nb = Tile<MM, X0, true, TT>::tiles(A.nx, A.ny);
            REQUIRE((size_t)(MM + 1) * (MM + 2) * nb <= c->partials_cap, "adjoint: reduction scratch too small");
            LAUNCH_NB(c, bytes, (k_gr_tile<T, MM, X0, TT>), dim3(nb), dim3(BLOCK), st, A.A, (const T*)A.px,
                      (const T*)A.py, (const C*)A.c0, (const C*)b, (const C*)x0, ko, 1.0 / tau(l), c->partials);
        };
        if (tt == 16) {
            if (x0) go(std::integral_constant<int, 16>{}, std::true_type{});
            else go(std::integral_constant<int, 16>{}, std::false_type{});
        } else {
            if (x0) go(std::integral_constant<int, 32>{}, std::true_type{});
            else go(std::integral_constant<int, 32>{}, std::false_type{});
        }
        return nb;
    }

    // rc (x0 = 0 only): also the restriction of the call's residual to the next level, from
    // the Krylov identity in the same pass as the combination.
    // rc: also rc = R (b - M x) (pre-smoother); pa_base, pa_out: also pa_out = pa_base + P x
    // on the finer level l - 1.
    void rec_gmres(int l, const void* b, const void* x0, int m, void* const* kv, GRec* R, void* xout,
                   void* rc = nullptr, const void* pa_base = nullptr, void* pa_out = nullptr) {
        AdrLevel& A = c->al[l];
        const size_t n = N(l);
        const int nb = fb(n);
        VecSet<T> K{};
        for (int q = 0; q <= m; ++q) K.v[q] = (const C*)kv[q];
        if (m <= 4) {
            int nt = 0;
            switch (m) {
                case 1: nt = rec_tile<1>(l, b, x0, kv); break;
                case 2: nt = rec_tile<2>(l, b, x0, kv); break;
                case 3: nt = rec_tile<3>(l, b, x0, kv); break;
                default: nt = rec_tile<4>(l, b, x0, kv); break;
            }
            const double sb = 8.0 * (m + 1) * (m + 2) * nt;
            switch (m) {
                case 1: LAUNCH_NB(c, sb, k_gr_solve_m<1>, dim3(1), dim3(SBLOCK), st, (const double*)c->partials, nt, R, tau(l)); break;
                case 2: LAUNCH_NB(c, sb, k_gr_solve_m<2>, dim3(1), dim3(SBLOCK), st, (const double*)c->partials, nt, R, tau(l)); break;
                case 3: LAUNCH_NB(c, sb, k_gr_solve_m<3>, dim3(1), dim3(SBLOCK), st, (const double*)c->partials, nt, R, tau(l)); break;
                default: LAUNCH_NB(c, sb, k_gr_solve_m<4>, dim3(1), dim3(SBLOCK), st, (const double*)c->partials, nt, R, tau(l)); break;
            }
            if (rc && !x0) {
                LAUNCH_NB(c, (m + 2.0) * sizeof(C) * n + sizeof(C) * n / 4.0, (k_gr_combine_rr<T>),
                          dim3(gr_rr_blocks(A.nx, A.ny)), dim3(BLOCK), st, A.nx, A.ny, K, m, (const GRec*)R, tau(l),
                          (C*)xout, (C*)rc);
                return;
            }
            if (pa_out) {
                LAUNCH_NB(c, (m + 1.0 + (x0 ? 1.0 : 0.0)) * sizeof(C) * n + 2.0 * sizeof(C) * 4.0 * n,
                          (k_gr_combine_pa<T>), dim3(gr_rr_blocks(2 * A.nx, 2 * A.ny)), dim3(BLOCK), st, A.nx, A.ny,
                          K, m, (const GRec*)R, (const C*)x0, (C*)xout, (const C*)pa_base, (C*)pa_out);
                return;
            }
            LAUNCH_NB(c, (m + 1.0 + (x0 ? 1.0 : 0.0)) * sizeof(C) * n, (k_gr_combine<T>), dim3(nb), dim3(BLOCK), st, n,
                      K, m, (const GRec*)R, (const C*)x0, (C*)xout);
            if (rc)
                LAUNCH(c, (3 * sizeof(C) + 2 * sizeof(T)) * NN2(A.nx, A.ny), (k_adr_resid_restrict<T>),
                       dim3(rr_blocks(A.nx, A.ny)), dim3(BLOCK), st, A.A, (const T*)A.px, (const T*)A.py,
                       (const C*)A.c0, (const C*)b, (const C*)xout, (C*)rc);
            return;
        }
        // the partials of k_{j+1} go to entries j (j + 1) .. (j + 1)(j + 2) - 1, the layout of
        // the record's Gram matrix, summed once by the solve
        REQUIRE((size_t)(m + 1) * (m + 2) * nb <= c->partials_cap, "adjoint: reduction scratch too small");
        LAUNCH_NB(c, (x0 ? 4.0 : 2.0) * sizeof(C) * n, (k_gr_r0<T>), dim3(nb), dim3(BLOCK), st, A.A, (const T*)A.px,
               (const T*)A.py, (const C*)A.c0, (const C*)b, (const C*)x0, (C*)kv[0], c->partials);
        for (int jj = 1; jj <= m; ++jj)
            LAUNCH_NB(c, (jj + 2.0) * sizeof(C) * n, (k_gr_chain<T>), dim3(nb), dim3(BLOCK), st, A.A, (const T*)A.px,
                   (const T*)A.py, (const C*)A.c0, K, jj, 1.0 / tau(l), (C*)kv[jj],
                   c->partials + (size_t)jj * (jj + 1) * nb);
        LAUNCH_NB(c, 8.0 * (m + 1) * (m + 2) * nb, k_gr_solve, dim3(1), dim3(FBLOCK), st, (const double*)c->partials,
               nb, R, tau(l));
        LAUNCH_NB(c, (m + 1.0 + (x0 ? 1.0 : 0.0)) * sizeof(C) * n, (k_gr_combine<T>), dim3(nb), dim3(BLOCK), st, n, K, m,
               (const GRec*)R, (const C*)x0, (C*)xout);
        if (rc)
            LAUNCH(c, (3 * sizeof(C) + 2 * sizeof(T)) * NN2(A.nx, A.ny), (k_adr_resid_restrict<T>),
                   dim3(rr_blocks(A.nx, A.ny)), dim3(BLOCK), st, A.A, (const T*)A.px, (const T*)A.py,
                   (const C*)A.c0, (const C*)b, (const C*)xout, (C*)rc);
        if (pa_out) {
            AdrLevel& F = c->al[l - 1];
            LAUNCH_NB(c, 2.25 * sizeof(C) * NN2(F.nx, F.ny), (k_prolong_copy<T>), dim3(tiles_of(F.nx, F.ny)),
                      tile_block(), st, F.nx, F.ny, (const C*)xout, (const C*)pa_base, (C*)pa_out);
        }
    }

    // ------------------------------------------------------------ reverse
    // fb[0] holds the cotangent of u_{k+1} on entry and that of u_k on exit.
    void rev_cycle(const void* g, const void* u0) {
        WaveLevel& W = c->wl[1];
        const Geom& G = W.G;
        const size_t NF = N(1);
        const int nb = fb(NF);
        LAUNCH_NB(c, (5.0 * sizeof(C) + sizeof(T)) * NF, (k_jacobi_adj<T>), dim3(nb), dim3(BLOCK), st, G, (const T*)W.n2,
               (const C*)g, (const C*)tp().uB, (const C*)S.fb[0], (C*)S.fb[1], T(c->w[0]), wslot());
        fin_add(nb, 0);
        restrict_adj(1, S.fb[1], S.lub[2]);
        rev_level(2);
        prolong_adj(1, S.lgb[2], S.fb[1], nullptr);
        LAUNCH_NB(c, ((u0 ? 5.0 : 4.0) * sizeof(C) + sizeof(T)) * NF, (k_jacobi_adj<T>), dim3(nb), dim3(BLOCK), st, G,
               (const T*)W.n2, (const C*)g, (const C*)u0, (const C*)S.fb[1], (C*)S.fb[0], T(c->w[0]), wslot());
        fin_add(nb, 0);
        wflush();
    }

    // out (level l+1) = 4 R x (level l): the cotangent of a coarse correction.
    void restrict_adj(int l, const void* x, void* out) {
        const int nx = c->wl[l].nx, ny = c->wl[l].ny;
        const size_t nc = N(l + 1);
        auto go = [&](auto tf, auto tc) {
            using Pf = decltype(tf);
            using Pc = decltype(tc);
            LAUNCH_NB(c, sizeof(cplx<Pf>) * NN2(nx, ny) + sizeof(cplx<Pc>) * double(nc), (k_restrict_scale<Pf, Pc>),
                   dim3(fb(nc)), dim3(BLOCK), st, nx, ny, (const cplx<Pf>*)x, (cplx<Pc>*)out, 4.0);
        };
        if (c->wl[l].f64) go(double{}, double{});
        else if (c->wl[l + 1].f64) go(T{}, double{});
        else go(T{}, T{});
    }
    // reverse of rc = R (g - A u) on level l: gbar += P rcbar/4, ubar -= A^H P rcbar/4
    void prolong_adj(int l, const void* rcbar, void* ubar, void* gbar) {
        WaveLevel& W = c->wl[l];
        const size_t n = N(l);
        auto go = [&](auto tf, auto tc) {
            using Pf = decltype(tf);
            using Pc = decltype(tc);
            LAUNCH_NB(c, (3.0 * sizeof(cplx<Pf>) + sizeof(Pf)) * n + sizeof(cplx<Pc>) * double(N(l + 1)),
                   (k_prolong_adj<Pc, Pf>), dim3(fb(n)), dim3(BLOCK), st, W.G, (const Pf*)W.n2,
                   (const cplx<Pc>*)rcbar, (cplx<Pf>*)ubar, (cplx<Pf>*)gbar);
        };
        if (W.f64) go(double{}, double{});
        else if (c->wl[l + 1].f64) go(T{}, double{});
        else go(T{}, T{});
    }

    // Reverse of m Chebyshev steps u' = u + q(N) A^H (g - A u) on level l (u == null:
    // from zero).  ubar holds u''s cotangent on entry and u's on exit; gbar += A q(N) ubar';
    // wacc[l-1] += Re <q_alpha(N) ubar', A^H (g - A u)>.
    template <typename P>
    void cheb_adj(int l, const void* g, const void* u, void* ubar, void* gbar, double alpha, int m) {
        using Cp = cplx<P>;
        WaveLevel& W = c->wl[l];
        const Geom& G = W.G;
        const size_t n = N(l);
        const int nb = fb(n);
        auto& B = S.cs[l];
        Cp *r = (Cp*)B[0], *rt = (Cp*)B[1], *d = (Cp*)B[2], *dt = (Cp*)B[3], *s = (Cp*)B[4], *stt = (Cp*)B[5];
        Cp *t1 = (Cp*)B[6], *t2 = (Cp*)B[7], *res = (Cp*)B[8];
        const double lam = W.lam;
        const double a = lam / alpha;
        const double th = 0.5 * (lam + a), dc = 0.5 * (lam - a);
        const double th_t = -lam / (2.0 * alpha * alpha), dc_t = lam / (2.0 * alpha * alpha);
        double rho = dc / th, rho_t = (dc_t * th - dc * th_t) / (th * th);
        LAUNCH_NB(c, 7.0 * sizeof(Cp) * n, (k_chebadj_start<P>), dim3(nb), dim3(BLOCK), st, n, (const Cp*)ubar, r, rt, d,
               dt, s, stt, P(1.0 / th), P(-th_t / (th * th)));
        // one fused pass per step; d, dt alternate with the buffers t1, t2
        for (int t = 1; t < m; ++t) {
            const double den = 2.0 * th - dc * rho;
            const double den_t = 2.0 * th_t - dc_t * rho - dc * rho_t;
            const double rn = dc / den, rn_t = (dc_t * den - dc * den_t) / (den * den);
            const double c1 = rn * rho, c1t = rn_t * rho + rn * rho_t;
            const double c2 = 2.0 / den, c2t = -2.0 * den_t / (den * den);
            LAUNCH_NB(c, (14.0 * sizeof(Cp) + sizeof(P)) * n, (k_chebadj_fused<P>), dim3(tiles_of(G.nx, G.ny)),
                      tile_block(), st, G, (const P*)W.n2, (const Cp*)d, (const Cp*)dt, t1, t2, r, rt, s, stt, P(c1),
                      P(c2), P(c1t), P(c2t));
            std::swap(d, t1);
            std::swap(dt, t2);
            rho = rn;
            rho_t = rn_t;
        }
        E.template residual<P>(G, W.n2, g, u, res);
        LAUNCH_NB(c, (2.0 * sizeof(Cp) + sizeof(P)) * n, (k_dot_ah<P>), dim3(nb), dim3(BLOCK), st, G, (const P*)W.n2,
               (const Cp*)stt, (const Cp*)res, wslot());
        fin_add(nb, l - 1);
        E.template applyA<P>(G, W.n2, s, t1, 0);
        LAUNCH_NB(c, (5.0 * sizeof(Cp) + sizeof(P)) * n, (k_adj_ahsub<P>), dim3(nb), dim3(BLOCK), st, G, (const P*)W.n2,
               (const Cp*)t1, (Cp*)(u ? ubar : nullptr), (Cp*)gbar);
    }

    void rev_level(int l) {
        WaveLevel& W = c->wl[l];
        const int L = c->L;
        const size_t n = N(l);
        prec(l, [&](auto tag) {
            using P = decltype(tag);
            E.template zero<P>(S.lgb[l], n);
        });
        if (l == L) {
            cheb_adj<double>(l, tp().g[l], nullptr, S.lub[l], S.lgb[l], c->w[l - 1], c->d.cheb_coarse);
            return;
        }
        if (l == 2 && S.M > 0) rev_adr_steps();
        if (l != 3 || c->d.level3_literal)
            cheb_adj<T>(l, tp().g[l], tp().ub[l], S.lub[l], S.lgb[l], c->w[l - 1], c->d.cheb_post);
        restrict_adj(l, S.lub[l], S.lub[l + 1]);
        rev_level(l + 1);
        prolong_adj(l, S.lgb[l + 1], l == 3 ? nullptr : S.lub[l], S.lgb[l]);
        if (l != 3) cheb_adj<T>(l, tp().g[l], nullptr, S.lub[l], S.lgb[l], c->w[l - 1], c->d.cheb_pre);
        (void)W;
    }

    // The ADR steps of level 2 in reverse: the last step's re-modulation, then per step the
    // reverse ADR V-cycle and one pass for its demodulation with the re-modulation of the
    // step before it.  The passes that produce a reverse call's xbar also form its dots
    // <k_j, xbar>.
    void rev_adr_steps() {
        WaveLevel& W = c->wl[2];
        const size_t n = N(2);
        const int M = S.M;
        int md = 0;
        VecSet<T> Kd = first_rev_basis(M - 1, 2, md);
        LAUNCH_NB(c, (3.0 * sizeof(C) + sizeof(T) + 16.0 + md * sizeof(C)) * n, (k_modadd_adj<T>), dim3(fb(n)),
                  dim3(BLOCK), st, n, (const C*)S.lub[2], (const C*)tp().adr[M - 1][2].xo, (const C*)c->car2,
                  (C*)S.axb[2], S.thb, Kd, md, c->partials);
        for (int s = M - 1; s >= 0; --s) {
            rev_adrv(s, 2);
            const C* an = s > 0 ? (const C*)tp().adr[s - 1][2].xo : nullptr;
            md = 0;
            Kd = s > 0 ? first_rev_basis(s - 1, 2, md) : VecSet<T>{};
            LAUNCH_NB(c, (8.0 * sizeof(C) + sizeof(T) + 16.0 + md * sizeof(C)) * n, (k_adr_step_adj<T>), dim3(fb(n)),
                      dim3(BLOCK), st, W.G, (const T*)W.n2, (const C*)S.abb[2], (const C*)tp().adr[s][2].b,
                      (const C*)c->car2, (C*)S.lub[2], (C*)S.lgb[2], S.thb, an, (C*)(an ? S.axb[2] : nullptr), Kd, md,
                      c->partials);
        }
    }

    // k_1..k_m of the first GMRES call that rev_adrv(s, l) reverses (the post-smoother of
    // level l, the only call on the coarsest level), m to md.
    VecSet<T> first_rev_basis(int s, int l, int& md) {
        AdrTape& Tp = tp().adr[s][l];
        md = gm_of(c, l);
        void* const* kv = l == c->LA ? Tp.kpre : Tp.kpost;
        VecSet<T> K{};
        for (int q = 0; q < md; ++q) K.v[q] = (const C*)kv[q];
        return K;
    }

    // Reverse of ADR V-cycle s from level l; its first reverse call finds the dots of its
    // xbar already in c->partials.
    void rev_adrv(int s, int l) {
        AdrTape& Tp = tp().adr[s][l];
        AdrLevel& A = c->al[l];
        const int m = gm_of(c, l);
        if (l == c->LA) {
            rev_gmres(l, nullptr, m, Tp.kpre, Tp.rpre, S.axb[l], S.abb[l], true, nullptr);
            return;
        }
        rev_gmres(l, Tp.x2, m, Tp.kpost, Tp.rpost, S.axb[l], S.abb[l], true, S.axb2[l]);
        const size_t nc = N(l + 1);
        int mc = 0;
        const VecSet<T> Kc = first_rev_basis(s, l + 1, mc);
        LAUNCH_NB(c, sizeof(C) * (double(N(l)) + nc * (1.0 + mc)), (k_restrict_scale_dots<T>), dim3(fb(nc)),
                  dim3(BLOCK), st, A.nx, A.ny, (const C*)S.axb2[l], (C*)S.axb[l + 1], 4.0, Kc, mc, c->partials);
        rev_adrv(s, l + 1);
        // the dots of the pre-smoother's reverse, <k_j, xbar>, come with this pass
        VecSet<T> Kd{};
        for (int q = 0; q < m; ++q) Kd.v[q] = (const C*)Tp.kpre[q];
        LAUNCH_NB(c, (6.0 * sizeof(C) + 2 * sizeof(T) + 32.0 * 2 + m * sizeof(C)) * NN2(A.nx, A.ny), (k_adr_rr_adj<T>),
                  dim3(fb(N(l))), dim3(BLOCK), st, A.A, (const T*)A.px, (const T*)A.py, (const C*)A.c0,
                  (const C*)S.abb[l + 1], (const C*)Tp.x1, (C*)S.axb2[l], (C*)S.abb[l], S.pxb[l], S.pyb[l], S.c0b[l],
                  Kd, m, c->partials);
        rev_gmres(l, nullptr, m, Tp.kpre, Tp.rpre, S.axb2[l], S.abb[l], false, nullptr);
    }

    // Reverse of x = GMRES(M_l; b, x0, m) from the recorded basis kv and record R:
    // bbar (=|+=) the cotangent of b; xbar0 (if x0) = that of x0.
    // The reverse of a recorded GMRES(MM) call's basis chain in one tile pass (k_ga_tile).
    template <int MM>
    void rev_tile(int l, const void* x0, const VecSet<T>& V, const GRec* R, void* bbar, bool bset, void* xbar0) {
        AdrLevel& A = c->al[l];
        constexpr int TT = 16;
        const int nt = ((A.nx - 2) / TT + 1) * ((A.ny - 2) / TT + 1);
        const double bytes = ((MM + 3.0 + (x0 ? 2.0 : 0.0) + (bset ? 0.0 : 1.0)) * sizeof(C) + 2 * sizeof(T) + 64.0) *
                             double(N(l));
        if (x0)
            LAUNCH_NB(c, bytes, (k_ga_tile<T, MM, true, TT>), dim3(nt), dim3(BLOCK), st, A.A, (const T*)A.px,
                      (const T*)A.py, (const C*)A.c0, V, (const double*)R->coef, 1.0 / tau(l), (const C*)x0, (C*)bbar,
                      bset ? 0 : 1, (C*)xbar0, S.pxb[l], S.pyb[l], S.c0b[l]);
        else
            LAUNCH_NB(c, bytes, (k_ga_tile<T, MM, false, TT>), dim3(nt), dim3(BLOCK), st, A.A, (const T*)A.px,
                      (const T*)A.py, (const C*)A.c0, V, (const double*)R->coef, 1.0 / tau(l), (const C*)nullptr,
                      (C*)bbar, bset ? 0 : 1, (C*)nullptr, S.pxb[l], S.pyb[l], S.c0b[l]);
    }

    // The partials of <k_j, xbar> (fb(N(l)) blocks) are already in c->partials: the pass
    // that produced xbar formed them.
    void rev_gmres(int l, const void* x0, int m, void* const* kv, GRec* R, const void* xbar, void* bbar, bool bset,
                   void* xbar0) {
        AdrLevel& A = c->al[l];
        const size_t n = N(l);
        const int nb = fb(n);
        const double pb = 16.0 * nb * m;
        switch (m) {
            case 1: LAUNCH_NB(c, pb, k_ga_prep_m<1>, dim3(1), dim3(SBLOCK), st, (const double*)c->partials, nb, R, tau(l)); break;
            case 2: LAUNCH_NB(c, pb, k_ga_prep_m<2>, dim3(1), dim3(SBLOCK), st, (const double*)c->partials, nb, R, tau(l)); break;
            case 3: LAUNCH_NB(c, pb, k_ga_prep_m<3>, dim3(1), dim3(SBLOCK), st, (const double*)c->partials, nb, R, tau(l)); break;
            case 4: LAUNCH_NB(c, pb, k_ga_prep_m<4>, dim3(1), dim3(SBLOCK), st, (const double*)c->partials, nb, R, tau(l)); break;
            default: LAUNCH_NB(c, pb, k_ga_prep, dim3(1), dim3(FBLOCK), st, (const double*)c->partials, nb, R, tau(l)); break;
        }
        VecSet<T> V{};
        V.v[0] = (const C*)xbar;
        for (int q = 0; q <= m; ++q) V.v[q + 1] = (const C*)kv[q];
        if (m <= 4) {
            switch (m) {
                case 1: rev_tile<1>(l, x0, V, R, bbar, bset, xbar0); break;
                case 2: rev_tile<2>(l, x0, V, R, bbar, bset, xbar0); break;
                case 3: rev_tile<3>(l, x0, V, R, bbar, bset, xbar0); break;
                default: rev_tile<4>(l, x0, V, R, bbar, bset, xbar0); break;
            }
            return;
        }
        const int nv = m + 2;
        C* acc = (C*)S.acc0[l];
        C* nxt = (C*)S.acc1[l];
        const double* coef = R->coef;
        const double gbytes = 32.0 * 2 + sizeof(C);  // coefficient cotangents (read-modify-write) and a
        LAUNCH_NB(c, (nv + 1.0) * sizeof(C) * n, (k_ga_step<T>), dim3(nb), dim3(BLOCK), st, A.A, (const T*)A.px,
               (const T*)A.py, (const C*)A.c0, V, nv, coef + m * GCOEF_STRIDE, (const C*)nullptr, 0.0,
               (const C*)nullptr, acc, S.pxb[l], S.pyb[l], S.c0b[l]);
        for (int j = m + 1; j >= 2; --j) {
            LAUNCH_NB(c, ((nv + 2.0) * sizeof(C) + 2 * sizeof(T)) * n + gbytes * n, (k_ga_step<T>), dim3(nb), dim3(BLOCK),
                   st, A.A, (const T*)A.px, (const T*)A.py, (const C*)A.c0, V, nv, coef + (j - 2) * GCOEF_STRIDE,
                   (const C*)acc, 1.0 / tau(l), (const C*)kv[j - 2], nxt, S.pxb[l], S.pyb[l], S.c0b[l]);
            std::swap(acc, nxt);
        }
        if (bset) copy(bbar, acc, n * sizeof(C));
        else LAUNCH(c, 3.0 * sizeof(C) * n, (k_axpy<T>), dim3(nb), dim3(BLOCK), st, n, T(1), (const C*)acc, (C*)bbar);
        if (x0) {
            VecSet<T> V1{};
            V1.v[0] = (const C*)xbar;
            LAUNCH_NB(c, (4.0 * sizeof(C) + 2 * sizeof(T)) * n + gbytes * n, (k_ga_step<T>), dim3(nb), dim3(BLOCK), st,
                   A.A, (const T*)A.px, (const T*)A.py, (const C*)A.c0, V1, 1, (const double*)R->one, (const C*)acc,
                   -1.0, (const C*)x0, (C*)xbar0, S.pxb[l], S.pyb[l], S.c0b[l]);
        }
    }

    // Cotangent of the fine phase from the accumulated coefficient cotangents.
    template <typename TO>
    void phase_out(void* grad_phi) {
        const int n = c->d.n;
        const size_t NF = N(1);
        if (S.M > 0) {
            for (int l = 2; l <= c->LA; ++l) {
                LAUNCH_NB(c, (2.0 * sizeof(T) + 32.0 + 16.0) * double(N(l)), (k_phi_adj<T>), dim3(fb(N(l))), dim3(BLOCK),
                       st, lnx(c, l), lny(c, l), 1 << (l - 2), n / 2, c->d.k, c->d.sign, (const T*)c->al[l].px,
                       (const T*)c->al[l].py,
                       (const double*)S.pxb[l], (const double*)S.pyb[l], (const c128*)S.c0b[l],
                       (const double*)(l == 2 ? S.thb : nullptr), S.phib2);
            }
            LAUNCH_NB(c, (sizeof(TO) + 2.0) * NF, (k_phi_out<TO>), dim3(fb(NF)), dim3(BLOCK), st, n, c->d.ny,
                   (const double*)S.phib2, (TO*)grad_phi);
        } else {
            HIPCHK(hipMemsetAsync(grad_phi, 0, NF * sizeof(TO), st));
        }
    }
};

// The checkpoint buffer of K cycles (library-owned unless ckpt_ws), u_0 (zero if NULL) in
// its first slot.
template <typename T>
static char* adj_checkpoints(helm_ctx c, int K, const void* u0, void* ckpt_ws, hipStream_t st) {
    if (!c->adj) c->adj = new AdjState();
    adj_alloc(c, st);
    AdjState& S = *c->adj;
    const size_t vb = (size_t)c->d.n * c->d.ny * sizeof(cplx<T>);
    char* ck = (char*)ckpt_ws;
    if (!ck) {
        if (S.ckpt_bytes < (size_t)K * vb) {
            dfree(c, S.ckpt);
            S.ckpt = nullptr;
            S.ckpt_bytes = 0;
            S.ckpt = dalloc(c, (size_t)K * vb);
            S.ckpt_bytes = (size_t)K * vb;
        }
        ck = (char*)S.ckpt;
    }
    if (u0) HIPCHK(hipMemcpyAsync(ck, u0, vb, hipMemcpyDeviceToDevice, st));
    else HIPCHK(hipMemsetAsync(ck, 0, vb, st));
    return ck;
}

// Zero accumulators of the coefficient, carrier, phase and weight cotangents, and the
// cotangent of u_K as the reverse sweep's start.
template <typename T>
static void adj_seed(helm_ctx c, const void* grad_uK, hipStream_t st) {
    AdjState& S = *c->adj;
    HIPCHK(hipMemsetAsync(S.wacc, 0, 64 * sizeof(double), st));
    if (S.M > 0) {
        for (int l = 2; l <= c->LA; ++l) {
            const size_t Nl = (size_t)lnx(c, l) * lny(c, l);
            HIPCHK(hipMemsetAsync(S.pxb[l], 0, Nl * sizeof(double), st));
            HIPCHK(hipMemsetAsync(S.pyb[l], 0, Nl * sizeof(double), st));
            HIPCHK(hipMemsetAsync(S.c0b[l], 0, Nl * sizeof(c128), st));
        }
        const size_t N2 = (size_t)lnx(c, 2) * lny(c, 2);
        HIPCHK(hipMemsetAsync(S.thb, 0, N2 * sizeof(double), st));
        HIPCHK(hipMemsetAsync(S.phib2, 0, N2 * sizeof(double), st));
    }
    HIPCHK(hipMemcpyAsync(S.fb[0], grad_uK, (size_t)c->d.n * c->d.ny * sizeof(cplx<T>), hipMemcpyDeviceToDevice,
                          st));
}

// Captures body on the capture stream into graph slot a (unless it holds a graph for the
// same key and K), then launches it on st.
template <typename T, typename Body>
static void adj_replay(helm_ctx c, AdjGraph& a, const void* k0, const void* k1, const void* k2, int K, hipStream_t st,
                       Body&& body) {
    if (!a.exec || a.key[0] != k0 || a.key[1] != k1 || a.key[2] != k2 || a.K != K) {
        if (a.exec) (void)hipGraphExecDestroy(a.exec);
        a = AdjGraph{};
        if (!c->cap_stream) HIPCHK(hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking));
        hipGraph_t graph = nullptr;
        HIPCHK(hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal));
        try {
            AdjEngine<T> Rc(c, c->cap_stream);
            body(Rc);
        } catch (...) {
            (void)hipStreamEndCapture(c->cap_stream, &graph);
            if (graph) (void)hipGraphDestroy(graph);
            throw;
        }
        HIPCHK(hipStreamEndCapture(c->cap_stream, &graph));
        hipGraphExec_t exec = nullptr;
        const hipError_t e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        HIPCHK(e);
        a.exec = exec;
        a.key[0] = k0;
        a.key[1] = k1;
        a.key[2] = k2;
        a.K = K;
    }
    HIPCHK(hipGraphLaunch(a.exec, st));
}

// The recording of K cycles from the checkpoint ck[0], one tape each; u_{k+1} from the
// recording into ck[k+1], and u_K into u_out when given.
template <typename T>
static void adj_record_all(AdjEngine<T>& E, const void* g, char* ck, int K, void* u_out) {
    AdjState& S = *E.c->adj;
    const size_t vb = (size_t)E.c->d.n * E.c->d.ny * sizeof(cplx<T>);
    for (int k = 0; k < K; ++k) {
        S.cur = k;
        E.rec_cycle(g, ck + (size_t)k * vb);
        if (k + 1 < K) E.post_jacobi(g, ck + (size_t)(k + 1) * vb);
        else if (u_out) E.post_jacobi(g, u_out);
    }
    S.cur = 0;
}

// The reverse sweep over K recorded tapes (u_k from the checkpoints).
template <typename T>
static void adj_reverse_all(AdjEngine<T>& E, const void* g, char* ck, int K) {
    AdjState& S = *E.c->adj;
    const size_t vb = (size_t)E.c->d.n * E.c->d.ny * sizeof(cplx<T>);
    for (int k = K - 1; k >= 0; --k) {
        S.cur = k;
        E.rev_cycle(g, ck + (size_t)k * vb);
    }
    S.cur = 0;
}

// The phase and weight cotangents from the accumulators.
template <typename T>
static void adj_finish(helm_ctx c, void* grad_phi, double* grad_w, hipStream_t st) {
    AdjEngine<T> R(c, st);
    if (c->f32) R.template phase_out<float>(grad_phi);
    else R.template phase_out<double>(grad_phi);
    HIPCHK(hipMemcpyAsync(grad_w, c->adj->wacc, c->L * sizeof(double), hipMemcpyDeviceToDevice, st));
}

// Checkpointed forward, then the reverse sweep over the K cycles.
template <typename T>
static void cycle_backward(helm_ctx c, int K, const void* g, const void* u0, const void* grad_uK, void* grad_phi,
                           double* grad_w, void* ckpt_ws, hipStream_t st) {
    char* ck = adj_checkpoints<T>(c, K, u0, ckpt_ws, st);
    AdjState& S = *c->adj;
    S.rec_valid = false;  // the tapes are rewritten here
    const size_t vb = (size_t)c->d.n * c->d.ny * sizeof(cplx<T>);
    adj_seed<T>(c, grad_uK, st);
    AdjEngine<T> R(c, st);
    const bool graphs = c->d.use_graphs && !c->prof.on;
    if (adj_tapes_for(c, K, st)) {
        // every cycle recorded once on its own tape, u_{k+1} from the recording, then the
        // reverse sweep over the tapes (about 1000 launches a cycle, one graph for all)
        auto body = [&](AdjEngine<T>& E) {
            adj_record_all<T>(E, g, ck, K, nullptr);
            adj_reverse_all<T>(E, g, ck, K);
        };
        if (graphs) adj_replay<T>(c, c->adj_graph[ADJ_FULL], g, ck, nullptr, K, st, body);
        else body(R);
    } else {
        // one tape: the K forward cycles for the checkpoints u_0 .. u_{K-1}, then per cycle
        // u_k into a fixed buffer, the recording and the reverse of that cycle, replayed
        // from one captured graph
        S.cur = 0;
        for (int k = 0; k + 1 < K; ++k) cycle_any(c, g, ck + (size_t)k * vb, ck + (size_t)(k + 1) * vb, st);
        for (int k = K - 1; k >= 0; --k) {
            const void* uk = ck + (size_t)k * vb;
            if (!graphs) {
                R.rec_cycle(g, uk);
                R.rev_cycle(g, uk);
                continue;
            }
            HIPCHK(hipMemcpyAsync(S.ubuf, uk, vb, hipMemcpyDeviceToDevice, st));
            adj_replay<T>(c, c->adj_graph[ADJ_FULL], g, ck, nullptr, 0, st, [&](AdjEngine<T>& E) {
                E.rec_cycle(g, S.ubuf);
                E.rev_cycle(g, S.ubuf);
            });
        }
    }
    adj_finish<T>(c, grad_phi, grad_w, st);
    HIPCHK(hipGetLastError());
}

// The forward half of a split adjoint: K cycles from u_0, each recorded on its own tape,
// u_K to u_out; false (nothing run) when the K tapes do not fit.
template <typename T>
static bool cycle_record(helm_ctx c, int K, const void* g, const void* u0, void* u_out, void* ckpt_ws,
                         hipStream_t st) {
    char* ck = adj_checkpoints<T>(c, K, u0, ckpt_ws, st);
    AdjState& S = *c->adj;
    S.rec_valid = false;
    if (!adj_tapes_for(c, K, st)) return false;
    const size_t vb = (size_t)c->d.n * c->d.ny * sizeof(cplx<T>);
    if (!S.uK) S.uK = dalloc(c, vb);
    // u_K goes to a buffer of the state, so that the graph does not depend on u_out
    auto body = [&](AdjEngine<T>& E) { adj_record_all<T>(E, g, ck, K, S.uK); };
    if (c->d.use_graphs && !c->prof.on) {
        adj_replay<T>(c, c->adj_graph[ADJ_REC], g, ck, nullptr, K, st, body);
    } else {
        AdjEngine<T> R(c, st);
        body(R);
    }
    HIPCHK(hipMemcpyAsync(u_out, S.uK, vb, hipMemcpyDeviceToDevice, st));
    HIPCHK(hipGetLastError());
    S.rec_valid = true;
    S.rec_K = K;
    S.rec_g = g;
    S.rec_ck = ck;
    S.rec_gen = c->data_gen;
    return true;
}

// The reverse half: the tapes of the last cycle_record, for the cotangent of its u_K.
template <typename T>
static void cycle_reverse(helm_ctx c, const void* grad_uK, void* grad_phi, double* grad_w, hipStream_t st) {
    AdjState& S = *c->adj;
    adj_seed<T>(c, grad_uK, st);
    auto body = [&](AdjEngine<T>& E) { adj_reverse_all<T>(E, S.rec_g, S.rec_ck, S.rec_K); };
    if (c->d.use_graphs && !c->prof.on) {
        adj_replay<T>(c, c->adj_graph[ADJ_REV], S.rec_g, S.rec_ck, nullptr, S.rec_K, st, body);
    } else {
        AdjEngine<T> R(c, st);
        body(R);
    }
    adj_finish<T>(c, grad_phi, grad_w, st);
    HIPCHK(hipGetLastError());
}

// L = ||g - A u||^2 (FP64) and, if grad_u, its cotangent -2 A^H (g - A u) in cycle precision.
template <typename T>
static double loss_grad(helm_ctx c, const void* g, const void* u, void* grad_u, hipStream_t st) {
    const Geom G = make_geom_sys(c);
    const size_t NF = (size_t)G.nx * G.ny;
    const int nb = flat_blocks(NF);
    LAUNCH_NB(c, (2.0 * sizeof(cplx<T>) + 8.0 + 16.0) * NF, (k_loss_resid<T>), dim3(nb), dim3(BLOCK), st, G,
           (const double*)c->n2f, (const cplx<T>*)g, (const cplx<T>*)u, (c128*)c->rbuf, c->partials);
    LAUNCH(c, 8.0 * nb, (k_finalize_sums<1>), dim3(1), dim3(FBLOCK), st, (const double*)c->partials, nb, 1, c->dscal);
    if (grad_u)
        LAUNCH_NB(c, (16.0 + 8.0 + sizeof(cplx<T>)) * NF, (k_loss_grad<T>), dim3(nb), dim3(BLOCK), st, G,
               (const double*)c->n2f, (const c128*)c->rbuf, (cplx<T>*)grad_u);
    double h = 0.0;
    HIPCHK(hipMemcpyAsync(&h, c->dscal, sizeof(double), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    return h;
}
