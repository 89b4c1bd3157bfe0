// Batched solves of independent problems of mixed sizes (the batch dimension of
// Section 1 and Section 4: many media solved together on one GPU).
//
// A native scheduler keeps `lanes` problems in flight: every lane is a host
// thread that drives its own HIP stream (default priority) and takes the next
// problem from a shared queue ordered by decreasing node count (longest first), so the
// small, launch-bound coarse levels of one problem overlap with the kernels of
// the others.  Every problem runs exactly the kernels and launch shapes of a
// single helm_solve on its own context, so its result equals the single solve
// bit for bit.  Per-problem convergence is tracked on the host (status, iters,
// relres); a converged problem leaves its lane to the next one.
//
// Included from helm.hip inside namespace helm.
#pragma once

// Runs job(p, lane) for p in `order` on `lanes` threads; each thread makes the
// batch's device current and uses its lane's stream.  Errors are returned per problem.
template <typename Job>
static void run_lanes(helm_batch b, const std::vector<int>& order, Job&& job, std::vector<helm_status>& st,
                      std::vector<std::string>& msg) {
    std::atomic<int> next{0};
    auto worker = [&](int lane) {
        const bool dev_ok = hipSetDevice(b->device) == hipSuccess;
        for (;;) {
            const int q = next.fetch_add(1);
            if (q >= (int)order.size()) break;
            const int p = order[q];
            if (!dev_ok) {
                st[p] = HELM_EHIP;
                msg[p] = "hipSetDevice failed on a lane thread";
                continue;
            }
            try {
                st[p] = job(p, lane);
            } catch (const Error& e) {
                st[p] = e.code;
                msg[p] = e.what();
            } catch (const std::exception& e) {
                st[p] = HELM_EHIP;
                msg[p] = e.what();
            } catch (...) {
                st[p] = HELM_EHIP;
                msg[p] = "unknown error";
            }
        }
    };
    std::vector<std::thread> th;
    for (int l = 1; l < b->lanes; ++l) th.emplace_back(worker, l);
    worker(0);
    for (auto& t : th) t.join();
}

// Runs job(j, lane) for j in [0, njobs) on the batch's lanes (jobs taken in order).
template <typename Job>
static void run_jobs(helm_batch b, int njobs, Job&& job) {
    std::atomic<int> next{0};
    auto worker = [&](int lane) {
        const bool dev_ok = hipSetDevice(b->device) == hipSuccess;
        for (;;) {
            const int q = next.fetch_add(1);
            if (q >= njobs) break;
            job(q, lane, dev_ok);
        }
    };
    std::vector<std::thread> th;
    for (int l = 1; l < b->lanes; ++l) th.emplace_back(worker, l);
    worker(0);
    for (auto& t : th) t.join();
}

static std::vector<int> longest_first_desc(const helm_desc* d, int np) {
    std::vector<int> order(np);
    for (int p = 0; p < np; ++p) order[p] = p;
    auto area = [&](int p) { return (size_t)d[p].n * (d[p].ny ? d[p].ny : d[p].n); };
    std::stable_sort(order.begin(), order.end(), [&](int a, int c) { return area(a) > area(c); });
    return order;
}

static std::vector<int> longest_first(helm_batch b) {
    std::vector<int> order(b->ctx.size());
    for (size_t p = 0; p < order.size(); ++p) order[p] = (int)p;
    auto area = [&](int p) { return (size_t)b->ctx[p]->d.n * b->ctx[p]->d.ny; };
    std::stable_sort(order.begin(), order.end(), [&](int a, int c) { return area(a) > area(c); });
    return order;
}

// Make every lane stream wait for the work queued so far on the caller's stream.
static void lanes_after(helm_batch b, hipStream_t caller) {
    HIPCHK(hipEventRecord(b->ev_in, caller));
    for (hipStream_t s : b->streams) HIPCHK(hipStreamWaitEvent(s, b->ev_in, 0));
}
// Make the caller's stream wait for everything queued on the lanes.
static void caller_after(helm_batch b, hipStream_t caller) {
    for (int l = 0; l < b->lanes; ++l) {
        HIPCHK(hipEventRecord(b->events[l], b->streams[l]));
        HIPCHK(hipStreamWaitEvent(caller, b->events[l], 0));
    }
}

static helm_status first_error(const std::vector<helm_status>& st, const std::vector<std::string>& msg) {
    helm_status worst = HELM_OK;
    for (size_t p = 0; p < st.size(); ++p) {
        if (st[p] == HELM_OK) continue;
        if (worst == HELM_OK || (worst == HELM_ENOCONV && st[p] != HELM_ENOCONV)) {
            worst = st[p];
            g_last_error = "problem " + std::to_string(p) + ": " +
                           (msg[p].empty() ? std::string(helm_status_string(st[p])) : msg[p]);
        }
    }
    return worst;
}

static void batch_free(helm_batch b) {
    if (!b) return;
    for (helm_ctx c : b->ctx)
        if (c) helm_destroy(c);
    for (auto& K : b->classes) {
        if (K.arena) (void)hipFree(K.arena);
        if (K.dg) (void)hipFree(K.dg);
        if (K.hg) (void)hipHostFree(K.hg);
        for (hipEvent_t e : K.ev)
            if (e) (void)hipEventDestroy(e);
    }
    for (hipStream_t s : b->streams) (void)hipStreamDestroy(s);
    for (hipEvent_t e : b->events) (void)hipEventDestroy(e);
    if (b->ev_in) (void)hipEventDestroy(b->ev_in);
    delete b;
}

// ------------------------------------------------------------------ lockstep classes
// Problems with equal descriptors (same n, levels, k, sponge, solver shape) form a class.
// Their contexts are built region by region in one arena: every device buffer of the
// q-th problem sits q * stride bytes after that of the first, so one launch with
// gridDim.z = P and the batch index {stride, p[z]} serves all of them (each kernel shifts
// its pointers by p[z] * stride).  The class then runs FP64 refinement around FP32
// FGMRES(restart) in lockstep: per iteration one launch per kernel for every problem
// still iterating, with each problem's own Krylov scalars, Givens rotations, stopping
// test and iteration count, so that each problem goes through exactly the operations of
// its single solve (helm_solve mode 1) and gives the same result bit for bit.
static constexpr int CLASS_GATHER = 2 * (MAXM + 2);  // doubles gathered per problem and column

static bool same_desc(const helm_desc& a, const helm_desc& b) { return std::memcmp(&a, &b, sizeof(helm_desc)) == 0; }

// The batch index of a launch over the problems `list` (region indices) of a class.
static void bset(helm_ctx c0, const std::vector<int>& list, size_t stride, const std::vector<int>* aux = nullptr) {
    BatchIdx bi{};
    bi.stride = (long long)stride;
    bi.n = (int)list.size();
    for (size_t z = 0; z < list.size(); ++z) {
        bi.p[z] = list[z];
        bi.aux[z] = aux ? (*aux)[z] : 0;
    }
    c0->bi = bi;
}

// Device bytes one problem of this descriptor allocates: its hierarchy, the inner bases of
// the refinement solve and the staging of g and u (measured by building it once).
static size_t class_stride(const helm_desc& d, const double* velocity, hipStream_t st) {
    helm_ctx c = new helm_ctx_s();
    c->d = desc_normalized(d);
    size_t bytes = 0;
    try {
        build(c, velocity, st);
        ensure_solver_ws(c, 1);
        c->bg = dalloc(c, (size_t)c->d.n * c->d.ny * sizeof(c128));
        c->bu = dalloc(c, (size_t)c->d.n * c->d.ny * sizeof(c128));
        bytes = c->count_bytes;
    } catch (...) {
        helm_destroy(c);
        throw;
    }
    helm_destroy(c);
    return (bytes + 65535) & ~size_t(65535);
}

// Builds problem p's context in region q of class K.
static helm_ctx class_build(helm_batch_s::Class& K, int q, const helm_desc& d, const double* velocity, const void* phi,
                            int phi_is_f64, hipStream_t st) {
    helm_ctx c = new helm_ctx_s();
    c->d = desc_normalized(d);
    c->arena = K.arena + (size_t)q * K.stride;
    c->arena_cap = K.stride;
    try {
        build(c, velocity, st);
        ensure_solver_ws(c, 1);
        c->bg = dalloc(c, (size_t)c->d.n * c->d.ny * sizeof(c128));
        c->bu = dalloc(c, (size_t)c->d.n * c->d.ny * sizeof(c128));
        REQUIRE(c->count_bytes <= K.stride, "batch class: a problem needs more device memory than its region");
        if (phi) set_phase(c, phi, phi_is_f64, st);
    } catch (...) {
        helm_destroy(c);
        throw;
    }
    return c;
}

// Whether class K can run in lockstep now: one phase per problem and equal launch shapes
// and weights (the launches are made from the first context's host state).
static bool class_lockstep_ok(helm_batch b, const helm_batch_s::Class& K) {
    if (K.probs.size() < 2 || !K.arena) return false;
    const helm_ctx c0 = b->ctx[K.probs[0]];
    for (int p : K.probs) {
        const helm_ctx c = b->ctx[p];
        if (c->nsets != 1 || !c->f32) return false;
        if (std::memcmp(&c->tn, &c0->tn, sizeof(c->tn)) != 0) return false;
        if (c->d.adr_steps > 0 && c->L >= 3 && !c->phase_set) return false;
    }
    return true;
}

// Gathers `count` doubles at src (an address inside region 0) for the problems of `list`
// into the class's pinned buffer (row z for list[z]); synchronous.
static const double* class_gather(helm_batch_s::Class& K, helm_ctx c0, const std::vector<int>& list, const double* src,
                                  int count, hipStream_t st) {
    bset(c0, list, K.stride);
    LAUNCH(c0, 0.0, k_gather, dim3(1), dim3(64), st, src, count, K.dg);
    HIPCHK(hipMemcpyAsync(K.hg, K.dg, sizeof(double) * count * list.size(), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    return K.hg;
}

// One restart cycle of the inner FP32 FGMRES for the problems `list` of class K (the
// class version of fgmres_cycle<float> with an unscaled preconditioner input, x = dbuf and
// a unit right-hand-side norm).  used[q], bd[q]: per region.
static void class_fgmres(helm_batch_s::Class& K, helm_ctx c0, const std::vector<int>& list,
                         const std::vector<double>& stop_abs, const std::vector<int>& maxit_left, std::vector<int>& used,
                         std::vector<char>& bd, hipStream_t st) {
    using Cp = c64;
    const int m = c0->d.restart;
    const Geom G = make_geom_sys(c0);
    const size_t N = (size_t)G.nx * G.ny;
    const size_t S = K.stride;
    KrylovScal* Kin = c0->Kin;
    const int nbf = c0->tn.fgmres_blocks > 0 ? std::min(c0->tn.fgmres_blocks, MAXRED) : flat_blocks(N, MAXRED);
    bset(c0, list, S);
    LAUNCH(c0, sizeof(Cp) * double(N), (k_krylov_init_norm<float>), dim3(nbf), dim3(BLOCK), st, N, (const Cp*)c0->iV[0],
           c0->partials);
    krylov_fin<MAXM>(c0, st, nbf, FIN_INIT, 0, m, Kin, 0.0);
    const double* hb = class_gather(K, c0, list, &Kin->beta, 1, st);
    const int P = (int)K.probs.size();
    std::vector<std::vector<std::vector<cd>>> H(P);
    std::vector<std::vector<double>> cs(P);
    std::vector<std::vector<cd>> sn(P), e(P);
    std::vector<int> jmax(P, 0);
    std::vector<int> run;
    for (size_t z = 0; z < list.size(); ++z) {
        const int q = list[z];
        const double beta = hb[z];
        used[q] = 0;
        bd[q] = 0;
        if (!(beta > 0.0) || !std::isfinite(beta)) {
            bd[q] = !std::isfinite(beta);
            continue;
        }
        H[q].assign(m + 1, std::vector<cd>(m, 0.0));
        cs[q].assign(m, 0.0);
        sn[q].assign(m, 0.0);
        e[q].assign(m + 1, 0.0);
        e[q][0] = beta;
        jmax[q] = std::min(m, maxit_left[q]);
        if (jmax[q] > 0) run.push_back(q);
    }
    VecSet<float> Vs{}, Zs{};
    for (int i = 0; i <= m; ++i) Vs.v[i] = (const Cp*)c0->iV[i];
    for (int i = 0; i < m; ++i) Zs.v[i] = (const Cp*)c0->iZ[i];
    std::vector<std::vector<int>> order(m + 1);  // problems of the enqueued iteration j
    const size_t cstride = (size_t)CLASS_GATHER;
    auto enqueue = [&](int j, const std::vector<int>& L) {
        order[j] = L;
        bset(c0, L, S);
        cycle_eager(c0, c0->iV[j], nullptr, c0->iZ[j], st);
        static_for_host<MAXM>(j, [&](auto jc) {
            constexpr int J = decltype(jc)::value;
            LAUNCH(c0, ((J + (J > 0 ? 4 : 3)) * sizeof(Cp) + sizeof(float)) * double(N), (k_fg_arnoldi<float, J>),
                   dim3(nbf), dim3(BLOCK), st, G, (const float*)c0->wl[1].n2, (const Cp*)c0->iZ[J], 1, Vs,
                   (Cp*)c0->iV[J], (Cp*)c0->iV[J + 1], (const KrylovScal*)Kin, c0->partials);
            krylov_fin<MAXM>(c0, st, nbf, FIN_LMV, J, m, Kin, 0.0);
            LAUNCH(c0, (J + 3) * sizeof(Cp) * double(N), (k_fg_orth<float, J>), dim3(nbf), dim3(BLOCK), st, N, Vs,
                   (Cp*)c0->iV[J + 1], (const KrylovScal*)Kin, c0->partials);
            krylov_fin<MAXM>(c0, st, nbf, FIN_LORTH, J, m, Kin, 0.0);
        });
        // column j of every problem of L into the pinned buffer (block j)
        LAUNCH(c0, 0.0, k_gather, dim3(1), dim3(64), st, (const double*)(Kin->H + 2 * (j * (MAXM + 1))), 2 * (j + 2),
               K.dg + (size_t)j * BMAX * cstride);
        HIPCHK(hipMemcpyAsync(K.hg + (size_t)j * BMAX * cstride, K.dg + (size_t)j * BMAX * cstride,
                              sizeof(double) * 2 * (j + 2) * L.size(), hipMemcpyDeviceToHost, st));
        HIPCHK(hipEventRecord(K.ev[j], st));
    };
    if (!run.empty()) enqueue(0, run);
    for (int j = 0; j < m && !run.empty(); ++j) {
        std::vector<int> next;
        for (int q : run)
            if (j + 1 < jmax[q]) next.push_back(q);
        if (!next.empty()) enqueue(j + 1, next);
        HIPCHK(hipEventSynchronize(K.ev[j]));
        const int cnt = 2 * (j + 2);
        std::vector<char> stop(P, 0);
        for (size_t z = 0; z < order[j].size(); ++z) {
            const int q = order[j][z];
            if (std::find(run.begin(), run.end(), q) == run.end()) continue;  // stopped before: speculative
            const double* col = K.hg + (size_t)j * BMAX * cstride + z * cnt;
            std::vector<std::vector<cd>>& Hq = H[q];
            for (int i = 0; i <= j + 1; ++i) Hq[i][j] = cd(col[2 * i], col[2 * i + 1]);
            const double hn = col[2 * (j + 1)];
            for (int i = 0; i < j; ++i) {
                cd t1 = cs[q][i] * Hq[i][j] + sn[q][i] * Hq[i + 1][j];
                cd t2 = -std::conj(sn[q][i]) * Hq[i][j] + cs[q][i] * Hq[i + 1][j];
                Hq[i][j] = t1;
                Hq[i + 1][j] = t2;
            }
            givens(Hq[j][j], Hq[j + 1][j], cs[q][j], sn[q][j]);
            Hq[j][j] = cs[q][j] * Hq[j][j] + sn[q][j] * Hq[j + 1][j];
            Hq[j + 1][j] = 0.0;
            e[q][j + 1] = -std::conj(sn[q][j]) * e[q][j];
            e[q][j] = cs[q][j] * e[q][j];
            used[q] = j + 1;
            const double est = std::abs(e[q][j + 1]);
            if (!std::isfinite(hn) || !std::isfinite(est)) {
                bd[q] = 1;
                stop[q] = 1;
            } else if (est < stop_abs[q] || hn == 0.0) {
                stop[q] = 1;
            }
        }
        std::vector<int> still;
        for (int q : next)
            if (!stop[q]) still.push_back(q);
        run = still;
    }
    // x += Z y for every problem with columns (its own count through the batch index)
    std::vector<int> act, cols;
    for (int q : list)
        if (used[q] > 0) {
            act.push_back(q);
            cols.push_back(used[q]);
        }
    if (!act.empty()) {
        bset(c0, act, S, &cols);
        LAUNCH(c0, 0.0, k_fgmres_lsq, dim3(1), dim3(64), st, Kin, -1);
        LAUNCH(c0, (m + 2) * sizeof(Cp) * double(N), (k_krylov_combine<float, MAXM>), dim3(flat_blocks(N)),
               dim3(BLOCK), st, N, Zs, (const KrylovScal*)Kin, (const Cp*)c0->dbuf, (Cp*)c0->dbuf, 1);
    }
    HIPCHK(hipStreamSynchronize(st));
}

// FP64 residual of the problems `list`: r into fV[0], sums into dscal; rn, gn per region.
static void class_residual(helm_batch_s::Class& K, helm_ctx c0, const std::vector<int>& list, std::vector<double>& rn,
                           std::vector<double>& gn, hipStream_t st) {
    const Geom G = make_geom_sys(c0);
    const int nbt = red_blocks(G.nx, G.ny);
    bset(c0, list, K.stride);
    LAUNCH(c0, (3 * 16.0 + 8.0 + 16.0) * NN2(G.nx, G.ny), k_residual_norms, dim3(nbt), tile_block(), st, G,
           (const double*)c0->n2f, (const c128*)c0->bg, (const c128*)c0->bu, (c128*)c0->fV[0], c0->partials);
    LAUNCH(c0, 16.0 * nbt, (k_finalize_sums<2>), dim3(1), dim3(FBLOCK), st, (const double*)c0->partials, nbt, 2,
           c0->dscal);
    const double* h = class_gather(K, c0, list, c0->dscal, 2, st);
    for (size_t z = 0; z < list.size(); ++z) {
        rn[list[z]] = std::sqrt(h[2 * z]);
        gn[list[z]] = std::sqrt(h[2 * z + 1]);
    }
}

// helm_solve mode 1 for every problem of class K in lockstep (see above).
static void class_solve(helm_batch b, helm_batch_s::Class& K, const void* const* g, void* const* u, double tol,
                        int maxit, int32_t* iters, double* relres, std::vector<helm_status>& st_out,
                        hipStream_t st) {
    const int P = (int)K.probs.size();
    helm_ctx c0 = b->ctx[K.probs[0]];
    const size_t NF = (size_t)c0->d.n * c0->d.ny;
    const size_t S = K.stride;
    for (int q = 0; q < P; ++q) {
        const helm_ctx c = b->ctx[K.probs[q]];
        HIPCHK(hipMemcpyAsync(c->bg, g[K.probs[q]], NF * sizeof(c128), hipMemcpyDeviceToDevice, st));
        HIPCHK(hipMemcpyAsync(c->bu, u[K.probs[q]], NF * sizeof(c128), hipMemcpyDeviceToDevice, st));
    }
    std::vector<double> rn(P, 0.0), gn(P, 0.0), r0(P, 0.0);
    std::vector<int> its(P, 0), used(P, 0);
    std::vector<char> bd(P, 0), done(P, 0);
    std::vector<helm_status> status(P, HELM_OK);
    std::vector<int> all(P);
    for (int q = 0; q < P; ++q) all[q] = q;
    class_residual(K, c0, all, rn, gn, st);
    std::vector<int> active;
    std::vector<int> zero;
    for (int q = 0; q < P; ++q) {
        if (!std::isfinite(gn[q]) || !std::isfinite(rn[q])) {
            status[q] = HELM_EBREAKDOWN;
            done[q] = 1;
        } else if (!(gn[q] > 0.0)) {
            zero.push_back(q);
            rn[q] = 0.0;
            gn[q] = 1.0;
            done[q] = 1;
        } else {
            r0[q] = rn[q];
            if (rn[q] / gn[q] < tol)
                done[q] = 1;
            else
                active.push_back(q);
        }
    }
    if (!zero.empty()) {
        bset(c0, zero, S);
        LAUNCH(c0, 16.0 * double(NF), (k_zero<double>), dim3(flat_blocks(NF)), dim3(BLOCK), st, NF, (c128*)c0->bu);
    }
    const double eta = 1e-4;
    while (!active.empty()) {
        bset(c0, active, S);
        LAUNCH(c0, 0.0, k_norm_scales, dim3(1), dim3(64), st, c0->dscal);
        LAUNCH(c0, 24.0 * double(NF), (k_cast_scale_dev<float, double>), dim3(flat_blocks(NF)), dim3(BLOCK), st, NF,
               (const c128*)c0->fV[0], (c64*)c0->iV[0], (const double*)c0->dscal + 2);
        LAUNCH(c0, 8.0 * double(NF), (k_zero<float>), dim3(flat_blocks(NF)), dim3(BLOCK), st, NF, (c64*)c0->dbuf);
        std::vector<double> target(P, 0.0);
        std::vector<int> left(P, 0);
        for (int q : active) {
            target[q] = std::max(eta, REFINE_MARGIN * tol * gn[q] / rn[q]);
            left[q] = maxit - its[q];
        }
        class_fgmres(K, c0, active, target, left, used, bd, st);
        bset(c0, active, S);
        LAUNCH(c0, 40.0 * double(NF), (k_add_cast_dev<double, float>), dim3(flat_blocks(NF)), dim3(BLOCK), st, NF,
               (const c64*)c0->dbuf, (c128*)c0->bu, (const double*)c0->dscal + 3);
        class_residual(K, c0, active, rn, gn, st);
        std::vector<int> still;
        for (int q : active) {
            its[q] += used[q];
            if (bd[q] || !std::isfinite(rn[q]) || rn[q] > 1e4 * r0[q]) {
                status[q] = HELM_EBREAKDOWN;
                continue;
            }
            const bool conv = rn[q] / gn[q] < tol;
            if (conv) continue;
            if (its[q] >= maxit || used[q] == 0) {
                status[q] = HELM_ENOCONV;
                continue;
            }
            still.push_back(q);
        }
        active = still;
    }
    for (int q = 0; q < P; ++q) {
        const int p = K.probs[q];
        const helm_ctx c = b->ctx[p];
        HIPCHK(hipMemcpyAsync(u[p], c->bu, NF * sizeof(c128), hipMemcpyDeviceToDevice, st));
        iters[p] = its[q];
        relres[p] = rn[q] / gn[q];
        st_out[p] = status[q];
    }
    c0->bi = BatchIdx{};
    HIPCHK(hipStreamSynchronize(st));
}
