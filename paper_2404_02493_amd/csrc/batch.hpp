// Batched solves of independent problems of mixed sizes (the batch dimension of
// Section 1 and Section 4: many media solved together on one GPU).
//
// A native scheduler keeps `lanes` problems in flight: every lane is a host
// thread that drives its own HIP stream (default priority) and takes the next
// problem from a shared queue ordered by decreasing n^2 (longest first), so the
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

static std::vector<int> longest_first_desc(const helm_desc* d, int np) {
    std::vector<int> order(np);
    for (int p = 0; p < np; ++p) order[p] = p;
    std::stable_sort(order.begin(), order.end(), [&](int a, int c) { return d[a].n > d[c].n; });
    return order;
}

static std::vector<int> longest_first(helm_batch b) {
    std::vector<int> order(b->ctx.size());
    for (size_t p = 0; p < order.size(); ++p) order[p] = (int)p;
    std::stable_sort(order.begin(), order.end(), [&](int a, int c) { return b->ctx[a]->d.n > b->ctx[c]->d.n; });
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
    for (hipStream_t s : b->streams) (void)hipStreamDestroy(s);
    for (hipEvent_t e : b->events) (void)hipEventDestroy(e);
    if (b->ev_in) (void)hipEventDestroy(b->ev_in);
    delete b;
}
