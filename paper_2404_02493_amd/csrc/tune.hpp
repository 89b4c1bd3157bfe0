// Autotuner of launch shapes, measured on the context's own hierarchy.
//
// Knobs (each changes only how the work and the FP64 partial sums of a reduction are
// split, hence only the summation order of those sums):
//   sstep_rows[l]    form of the s-step GMRES passes on ADR level l: steps per
//                    marching unit (rows of the unit plus its warm-up rows; longer
//                    units recompute fewer warm-up rows and leave fewer partials to
//                    sum, shorter ones give more wavefronts), or 1 / 2 for the
//                    overlapped-tile form with 16 x 16 / 32 x 32 tiles (more
//                    parallelism on small levels, more recomputed ring nodes);
//   fgmres_blocks    blocks of the outer FGMRES passes on the fine grid.
// Every candidate runs the real kernels on the level's buffers filled with
// hashed data; the fastest (HIP-event time over a few repetitions) is kept.  The
// result is a small JSON text that helm_set_tuning applies again later, so a
// caller can cache it per (device, problem size, precision).
//
// Included from helm.hip inside namespace helm.
#pragma once

// x = hashed values in [-1, 1] + i [-1, 1] on the unknowns, 0 on the ring.
template <typename T>
__global__ __launch_bounds__(BLOCK) void k_fill_hash(int n, int ny, uint32_t seed, cplx<T>* __restrict__ x) {
    const size_t N = (size_t)n * ny;  // n nodes per row, ny rows
    for (size_t p = blockIdx.x * (size_t)BLOCK + threadIdx.x; p < N; p += (size_t)gridDim.x * BLOCK) {
        const int i = (int)(p / n), j = (int)(p % n);
        uint64_t h = (uint64_t)p * 0x9E3779B97F4A7C15ull + seed;
        h ^= h >> 31;
        h *= 0xBF58476D1CE4E5B9ull;
        h ^= h >> 29;
        const double a = double(h & 0xFFFFFF) / double(0x800000) - 1.0;
        const double b = double((h >> 24) & 0xFFFFFF) / double(0x800000) - 1.0;
        x[p] = (i == 0 || j == 0) ? cplx<T>{} : mk<T>(T(a), T(b));
    }
}

// A Krylov state that lets the FGMRES passes run with every coefficient zero.
__global__ void k_tune_kstate(KrylovScal* K) {
    if (threadIdx.x != 0) return;
    K->done = 0;
    K->beta = 1.0;
    for (int i = 0; i <= MAXM; ++i) K->scale[i] = K->zscale[i] = 1.0;
    for (int i = 0; i < 2 * (MAXM + 2); ++i) K->dots[i] = 0.0;
}

template <typename F>
static double time_ms(hipStream_t st, int reps, F&& f) {
    hipEvent_t a, b;
    HIPCHK(hipEventCreate(&a));
    HIPCHK(hipEventCreate(&b));
    f();  // warm
    HIPCHK(hipEventRecord(a, st));
    for (int r = 0; r < reps; ++r) f();
    HIPCHK(hipEventRecord(b, st));
    HIPCHK(hipEventSynchronize(b));
    float ms = 0.f;
    HIPCHK(hipEventElapsedTime(&ms, a, b));
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    return double(ms) / reps;
}

static std::string tuning_json(helm_ctx c, const std::string& timings) {
    std::string out = "{\"n\": " + std::to_string(c->d.n) +
                      (c->d.ny != c->d.n ? ", \"ny\": " + std::to_string(c->d.ny) : std::string()) +
                      ", \"levels\": " + std::to_string(c->L) +
                      ", \"prec\": \"" + (c->f32 ? "c64" : "c128") + "\", \"sstep_rows\": {";
    bool first = true;
    for (int l = 2; l <= c->LA && l < 16; ++l) {
        if (c->tn.sstep_rows[l] <= 0) continue;
        out += std::string(first ? "" : ", ") + "\"" + std::to_string(l) + "\": " + std::to_string(c->tn.sstep_rows[l]);
        first = false;
    }
    out += "}, \"fgmres_blocks\": " + std::to_string(c->tn.fgmres_blocks);
    if (!timings.empty()) out += ", \"timings_ms\": {" + timings + "}";
    return out + "}";
}

template <typename T>
static std::string tune_ctx(helm_ctx c, hipStream_t st) {
    Engine<T> E(c, st);
    char buf[128];
    std::string tim;
    auto note = [&](const std::string& key, double ms) {
        std::snprintf(buf, sizeof(buf), "%s\"%s\": %.5f", tim.empty() ? "" : ", ", key.c_str(), ms);
        tim += buf;
    };
    const int reps = 5;
    // ADR levels that run the s-step form
    // (coarsest level first, so that every level is timed inside what surrounds it in the
    // cycle: a level below 2 as its V-cycle adding its prolongation into the next finer
    // level, the fused tile epilogues included; level 2 as two ADR correction steps)
    if (c->L >= 3 && c->d.adr_steps > 0 && !c->d.gmres_arnoldi) {
        for (int l = std::min(c->LA, 15); l >= 2; --l) {
            AdrLevel& A = c->al[l];
            const int m = l == c->LA ? c->d.gmres_coarse_m : c->d.gmres_m;
            if (m > 4) continue;
            if (E.block_form(l, m)) continue;  // one-workgroup form
            const int nb = flat_blocks((size_t)A.nx * A.ny);
            hipLaunchKernelGGL((k_fill_hash<T>), dim3(nb), dim3(BLOCK), 0, st, A.nx, A.ny, 17u + l, (cplx<T>*)A.b);
            hipLaunchKernelGGL((k_fill_hash<T>), dim3(nb), dim3(BLOCK), 0, st, A.nx, A.ny, 91u + l, (cplx<T>*)A.x);
            if (l == 2) {
                WaveLevel& W = c->wl[2];
                hipLaunchKernelGGL((k_fill_hash<T>), dim3(nb), dim3(BLOCK), 0, st, W.nx, W.ny, 23u, (cplx<T>*)W.g);
                hipLaunchKernelGGL((k_fill_hash<T>), dim3(nb), dim3(BLOCK), 0, st, W.nx, W.ny, 29u, (cplx<T>*)W.u);
            }
            HIPCHK(hipGetLastError());
            int best = 0;
            double tbest = 1e30;
            for (int cand : {1, 2, 16, 24, 32, 40, 48, 64, 80, 96, 128}) {
                if (cand > 16 && cand >= 2 * A.ny) break;  // segments run down the rows
                c->tn.sstep_rows[l] = cand;
                const double t = time_ms(st, reps, [&] {
                    if (l > 2) {
                        E.adr_vcycle(l, EPI_X, nullptr, c->al[l - 1].x);
                    } else if (c->phase_set) {
                        E.adr_steps(2);
                    } else {  // no carrier yet: the smoother pair alone
                        E.gmres(l, m, true);
                        E.gmres(l, m, false);
                    }
                });
                note("sstep_l" + std::to_string(l) + "_" + (cand == 1 ? std::string("tile16") : cand == 2 ? std::string("tile32") : std::to_string(cand)), t);
                if (t < tbest) {
                    tbest = t;
                    best = cand;
                }
            }
            c->tn.sstep_rows[l] = best;
        }
    }
    // outer FGMRES passes on the fine grid (basis of the inner solver for complex64
    // cycles, of the FP64 solver otherwise), at the middle of a restart cycle
    {
        const int mode = c->f32 ? 1 : 0;
        ensure_solver_ws(c, mode);
        const Geom G = make_geom_sys(c);
        const size_t NF = (size_t)G.nx * G.ny;
        const int jj = std::max(0, c->d.restart / 2);
        void** Vp = c->f32 ? c->iV : c->fV;
        void** Zp = c->f32 ? c->iZ : c->fZ;
        const void* n2 = c->f32 ? c->wl[1].n2 : (const void*)c->n2f;
        for (int i = 0; i <= jj + 1; ++i)
            hipLaunchKernelGGL((k_fill_hash<T>), dim3(flat_blocks(NF)), dim3(BLOCK), 0, st, G.nx, G.ny, 1000u + i,
                               (cplx<T>*)Vp[i]);
        hipLaunchKernelGGL((k_fill_hash<T>), dim3(flat_blocks(NF)), dim3(BLOCK), 0, st, G.nx, G.ny, 7u,
                           (cplx<T>*)Zp[0]);
        hipLaunchKernelGGL(k_tune_kstate, dim3(1), dim3(64), 0, st, c->Kin);
        HIPCHK(hipGetLastError());
        VecSet<T> Vs{};
        for (int i = 0; i <= c->d.restart; ++i) Vs.v[i] = (const cplx<T>*)Vp[i];
        int best = 0;
        double tbest = 1e30;
        for (int cand = 256; cand <= MAXRED; cand *= 2) {
            const double t = time_ms(st, reps, [&] {
                static_for_host<MAXM>(jj, [&](auto jc) {
                    constexpr int J = decltype(jc)::value;
                    hipLaunchKernelGGL((k_fg_arnoldi<T, J>), dim3(cand), dim3(BLOCK), 0, st, G, (const T*)n2,
                                       (const cplx<T>*)Zp[0], 0, Vs, (cplx<T>*)Vp[J], (cplx<T>*)Vp[J + 1],
                                       (const KrylovScal*)c->Kin, c->partials, BatchIdx{});
                    hipLaunchKernelGGL((k_fg_orth<T, J>), dim3(cand), dim3(BLOCK), 0, st, NF, Vs,
                                       (cplx<T>*)Vp[J + 1], (const KrylovScal*)c->Kin, c->partials, BatchIdx{});
                });
            });
            HIPCHK(hipGetLastError());
            note("fgmres_" + std::to_string(cand), t);
            if (t < tbest) {
                tbest = t;
                best = cand;
            }
        }
        c->tn.fgmres_blocks = best;
    }
    HIPCHK(hipStreamSynchronize(st));
    drop_graphs(c);
    return tuning_json(c, tim);
}

// Applies {"sstep_rows": {"l": steps or tile form, ...}, "fgmres_blocks": blocks} (other keys ignored).
static void apply_tuning(helm_ctx c, const char* json) {
    const std::string s(json);
    helm_ctx_s::Tuning t = c->tn;
    auto skip_ws = [&](size_t& i) {
        while (i < s.size() && (s[i] == ' ' || s[i] == '\n' || s[i] == '\t' || s[i] == '\r')) ++i;
    };
    auto read_int = [&](size_t& i) -> long {
        skip_ws(i);
        REQUIRE(i < s.size() && (std::isdigit((unsigned char)s[i]) || s[i] == '-'), "tuning: integer expected");
        size_t used = 0;
        long v = std::stol(s.substr(i), &used);
        i += used;
        return v;
    };
    size_t k = s.find("\"sstep_rows\"");
    if (k != std::string::npos) {
        size_t i = s.find('{', k);
        REQUIRE(i != std::string::npos, "tuning: sstep_rows must be an object");
        ++i;
        for (int l = 0; l < 16; ++l) t.sstep_rows[l] = 0;
        for (;;) {
            skip_ws(i);
            REQUIRE(i < s.size(), "tuning: unterminated sstep_rows");
            if (s[i] == '}') break;
            if (s[i] == ',') {
                ++i;
                continue;
            }
            REQUIRE(s[i] == '"', "tuning: level key expected");
            ++i;
            const long l = read_int(i);
            REQUIRE(i < s.size() && s[i] == '"', "tuning: level key expected");
            ++i;
            skip_ws(i);
            REQUIRE(i < s.size() && s[i] == ':', "tuning: ':' expected");
            ++i;
            const long v = read_int(i);
            REQUIRE(l >= 2 && l <= c->LA && l < 16, "tuning: level out of range");
            REQUIRE(v == 0 || v == 1 || v == 2 || (v >= 16 && v <= 256 && v % 8 == 0),
                    "tuning: unit steps out of range");
            t.sstep_rows[l] = (int)v;
        }
    }
    k = s.find("\"fgmres_blocks\"");
    if (k != std::string::npos) {
        size_t i = s.find(':', k);
        REQUIRE(i != std::string::npos, "tuning: fgmres_blocks value expected");
        ++i;
        const long v = read_int(i);
        REQUIRE(v >= 0 && v <= MAXRED, "tuning: block count out of range");
        t.fgmres_blocks = (int)v;
    }
    c->tn = t;
    drop_graphs(c);
}
