// helm_eikonal: travel-time phase of point sources on the device (factored eikonal
// equation, Section 3.2.1) installed as the phase of the ADR correction.
//
// Included from helm.hip after the phase-set helpers.
#pragma once

// ADR coefficients of every ADR level and the level-2 carrier from tau1 of one source
// (product-rule derivatives), into the current phase set.
static void build_phase_factored(helm_ctx c, const double* tau1, double xs, double ys, hipStream_t st) {
    for (int l = 2; l <= c->LA; ++l) {
        AdrLevel& A = c->al[l];
        const Geom G = make_geom(c, l);
        const int nb = flat_blocks((size_t)A.nx * A.ny);
        void* th = (l == 2) ? c->car2 : nullptr;
        if (c->f32)
            hipLaunchKernelGGL((k_adr_coef_fac<float>), dim3(nb), dim3(BLOCK), 0, st, G, (const double*)c->n2f, tau1, xs,
                               ys, c->d.k, c->d.sign, c->d.damping_strength, (float*)A.px, (float*)A.py, (c64*)A.c0,
                               (c64*)th);
        else
            hipLaunchKernelGGL((k_adr_coef_fac<double>), dim3(nb), dim3(BLOCK), 0, st, G, (const double*)c->n2f, tau1,
                               xs, ys, c->d.k, c->d.sign, c->d.damping_strength, (double*)A.px, (double*)A.py,
                               (c128*)A.c0, (c128*)th);
    }
    HIPCHK(hipGetLastError());
}

// Device buffers of one helm_eikonal call (freed on every exit path).
struct EikBufs {
    double* s = nullptr;
    double* t1 = nullptr;
    double* phi = nullptr;
    double* part = nullptr;
    double* mx = nullptr;
    double* host = nullptr;  // pinned: the round's largest decrease
    ~EikBufs() {
        (void)hipFree(s);
        (void)hipFree(t1);
        (void)hipFree(phi);
        (void)hipFree(part);
        (void)hipFree(mx);
        (void)hipHostFree(host);
    }
};

// Fills x[0..N) with v.
__global__ __launch_bounds__(BLOCK) void k_eik_fill(size_t N, double v, double* __restrict__ x) {
    for (size_t p = blockIdx.x * (size_t)BLOCK + threadIdx.x; p < N; p += (size_t)gridDim.x * BLOCK) x[p] = v;
}

// One round (four passes); a pass is one launch per anti-diagonal d of the Ty x Tx tiles
// (I + J = d, I < Ty rows, J < Tx columns).
template <int B>
static void eik_round(const EikSrc& E, const double* s, double* t1, double* part, hipStream_t st) {
    const int Tx = E.nx / B, Ty = E.ny / B;
    for (int pass = 0; pass < 4; ++pass) {
        const int iup = pass < 2 ? 1 : 0, jup = (pass % 2) == 0 ? 1 : 0;
        for (int d = 0; d <= Tx + Ty - 2; ++d) {
            const int lo = std::max(0, d - Tx + 1), hi = std::min(d, Ty - 1);
            hipLaunchKernelGGL((k_eik_pass<B>), dim3(hi - lo + 1), dim3(B), 0, st, E, s, t1, iup, jup, d, part);
        }
    }
}

// Returns HELM_ENOCONV (phase unchanged) if a node is still unreached after max_rounds.
static helm_status eikonal(helm_ctx c, const double* src, int nsrc, int max_rounds, double tol, void* tau1_out,
                           void* phi_out, int* rounds_out, double* change_out, hipStream_t st) {
    const int n = c->d.n, ny = c->d.ny;  // nodes per row, rows
    const double h = 1.0 / std::max(n, ny);
    REQUIRE(src != nullptr, "helm_eikonal: src_xy is NULL");
    REQUIRE(nsrc >= 1 && nsrc <= 64, "helm_eikonal: nsrc must be in 1..64");
    REQUIRE(max_rounds >= 1 && max_rounds <= 100000, "helm_eikonal: max_rounds must be in 1..100000");
    REQUIRE(!std::isnan(tol), "helm_eikonal: tol is NaN");
    for (int q = 0; q < nsrc; ++q) {
        const double x = src[2 * q], y = src[2 * q + 1];
        REQUIRE(x >= 0.0 && x <= double(n - 1) * h && y >= 0.0 && y <= double(ny - 1) * h,
                "helm_eikonal: sources must lie in [0, (n-1) h] x [0, (ny-1) h]");
    }
    const size_t NF = (size_t)n * ny;
    const int B = std::min(64, std::min(n, ny));  // divides both (powers of two)
    const size_t NT = (size_t)(n / B) * (ny / B);  // tiles
    EikBufs b;
    HIPCHK(hipMalloc((void**)&b.s, NF * sizeof(double)));
    HIPCHK(hipMalloc((void**)&b.t1, NF * sizeof(double)));
    HIPCHK(hipMalloc((void**)&b.phi, NF * sizeof(double)));
    HIPCHK(hipMalloc((void**)&b.part, NT * sizeof(double)));
    HIPCHK(hipMalloc((void**)&b.mx, 2 * sizeof(double)));
    HIPCHK(hipHostMalloc((void**)&b.host, 2 * sizeof(double), hipHostMallocDefault));
    hipLaunchKernelGGL(k_eik_slowness, dim3(flat_blocks(NF)), dim3(BLOCK), 0, st, NF, (const double*)c->n2f, b.s);
    hipLaunchKernelGGL(k_eik_fill, dim3(flat_blocks(NF)), dim3(BLOCK), 0, st, NF, __builtin_huge_val(), b.phi);
    HIPCHK(hipGetLastError());
    int rounds_max = 0;
    double change_max = 0.0;
    for (int q = 0; q < nsrc; ++q) {
        EikSrc E{n, ny, h, src[2 * q], src[2 * q + 1], std::sqrt(2.0) * h};
        long in = (long)std::floor(E.ys / h + 0.5), jn = (long)std::floor(E.xs / h + 0.5);
        in = std::min<long>(std::max<long>(in, 0), ny - 1);
        jn = std::min<long>(std::max<long>(jn, 0), n - 1);
        hipLaunchKernelGGL(k_eik_init, dim3(flat_blocks(NF)), dim3(BLOCK), 0, st, E, (const double*)b.s,
                           (size_t)in * n + jn, b.t1);
        int done = 0;
        double last = __builtin_huge_val();
        while (done < max_rounds) {
            hipLaunchKernelGGL(k_eik_fill, dim3(1), dim3(BLOCK), 0, st, NT, 0.0, b.part);
            if (B == 64) eik_round<64>(E, b.s, b.t1, b.part, st);
            else if (B == 32) eik_round<32>(E, b.s, b.t1, b.part, st);
            else eik_round<16>(E, b.s, b.t1, b.part, st);
            hipLaunchKernelGGL(k_eik_max, dim3(1), dim3(1024), 0, st, NT, (const double*)b.part, b.mx);
            HIPCHK(hipGetLastError());
            HIPCHK(hipMemcpyAsync(b.host, b.mx, sizeof(double), hipMemcpyDeviceToHost, st));
            HIPCHK(hipStreamSynchronize(st));
            ++done;
            last = b.host[0];
            if (tol >= 0.0 && last <= tol) break;
        }
        // a node still at +inf was never reached
        hipLaunchKernelGGL(k_eik_max, dim3(1), dim3(1024), 0, st, NF, (const double*)b.t1, b.mx);
        HIPCHK(hipGetLastError());
        HIPCHK(hipMemcpyAsync(b.host, b.mx, sizeof(double), hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
        if (!(b.host[0] < __builtin_huge_val())) {
            g_last_error = "helm_eikonal: nodes not reached within max_rounds";
            if (rounds_out) *rounds_out = done;
            if (change_out) *change_out = last;
            return HELM_ENOCONV;
        }
        hipLaunchKernelGGL(k_eik_phase, dim3(flat_blocks(NF)), dim3(BLOCK), 0, st, E, (const double*)b.t1, b.phi);
        HIPCHK(hipGetLastError());
        rounds_max = std::max(rounds_max, done);
        change_max = std::max(change_max, last);
    }
    if (c->L >= 3) {
        use_set(c, 0);
        c->nsets = 1;
        if (nsrc == 1)
            build_phase_factored(c, b.t1, src[0], src[1], st);
        else
            build_phase(c, b.phi, 1, st);
    }
    if (tau1_out) HIPCHK(hipMemcpyAsync(tau1_out, b.t1, NF * sizeof(double), hipMemcpyDeviceToDevice, st));
    if (phi_out) HIPCHK(hipMemcpyAsync(phi_out, b.phi, NF * sizeof(double), hipMemcpyDeviceToDevice, st));
    HIPCHK(hipStreamSynchronize(st));
    drop_graphs(c);
    c->phase_set = true;
    c->phase_factored = nsrc == 1 && c->L >= 3;
    ++c->data_gen;
    if (rounds_out) *rounds_out = rounds_max;
    if (change_out) *change_out = change_max;
    return HELM_OK;
}
