/*
 * Factored eikonal equation, oracle (test infrastructure only: the tests and the
 * benchmark's CPU leg call it; the library never does).
 *
 * Section 3.2.1 writes the travel time as tau = tau0 * tau1 with
 * tau0 = |x - x0| (the exact solution for unit slowness, eq. eikonal_cons), so
 * that tau1 solves |tau0 grad tau1 + tau1 grad tau0|^2 = s^2 and stays smooth at
 * the source.  The paper does not print a discretisation; the one used here is
 * the first-order upwind (Godunov) form of that equation on the stored nodes, nx
 * columns and ny rows (x = j h, y = i h), with grad tau0 exact:
 *
 *   per axis, the neighbour with the smaller tau = tau0 tau1 is the upwind one q;
 *   with sgn = +1 for the west / south neighbour and -1 for the east / north one,
 *     d tau / dx  ~  a_x t - b_x,   a_x = sgn r / h + g_x,   b_x = sgn r tau1(q) / h,
 *   r = tau0 at the node, g = grad tau0 = (x - x0) / r, t = tau1 at the node.
 *   This is the Godunov upwind scheme of |grad tau| = s with those one-sided
 *   differences.  Candidates: both axes, (a_x t - b_x)^2 + (a_y t - b_y)^2 = s^2,
 *   its larger root, kept when it is real and upwind on both axes
 *   (sgn (a t - b) >= 0); and one axis alone, sgn_x (a_x t - b_x) = s (no slope of
 *   tau along the other axis), likewise in y.  The update is the smallest
 *   candidate, and tau1 only decreases.
 *
 * Nodes within sqrt(2) h of the source are fixed at tau1 = (s(node) + s(src)) / 2,
 * s(src) the slowness at the node nearest the source (the straight-ray value,
 * exact for a constant medium); every other node starts at +infinity.
 *
 * oracle_eik_sweep solves that discrete system by fast sweeping: Gauss-Seidel
 * passes in the orders (i up, j up), (i up, j down), (i down, j up),
 * (i down, j down); one round is those four passes; rounds repeat until the
 * largest single decrease of tau1 in a round is at most tol (tol < 0: exactly
 * max_rounds rounds).
 *
 * Every operation is a single IEEE double operation (compile without contraction,
 * -ffp-contract=off), so that another implementation of the same steps can be
 * compared bit for bit.  Layout: row-major, index i nx + j.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>

typedef struct {
    int64_t nx, ny;
    double h, xs, ys;
    const double *s;
} eik_t;

static double node_r(const eik_t *E, int64_t i, int64_t j) {
    const double dx = (double)j * E->h - E->xs;
    const double dy = (double)i * E->h - E->ys;
    return sqrt(dx * dx + dy * dy);
}

/* the larger root of A t^2 - 2 B t + C = 0; returns 0 if there is no real root */
static int big_root(double A, double B, double C, double *t) {
    if (!(A > 0.0)) return 0;
    const double disc = B * B - A * C;
    if (!(disc >= 0.0)) return 0;
    *t = (B + sqrt(disc)) / A;
    return 1;
}

/* New tau1 at (i, j) from the current values T (tau1), or +inf if no candidate. */
static double local_update(const eik_t *E, const double *T, int64_t i, int64_t j) {
    const int64_t n = E->nx, ny = E->ny;
    const double h = E->h;
    const double x = (double)j * h, y = (double)i * h;
    const double dx = x - E->xs, dy = y - E->ys;
    const double r = sqrt(dx * dx + dy * dy);
    const double gx = dx / r, gy = dy / r;
    const double sp = E->s[i * n + j];
    /* upwind neighbour per axis */
    int hx = 0, hy = 0;
    double tqx = INFINITY, tqy = INFINITY, ux = 0.0, uy = 0.0, sgx = 0.0, sgy = 0.0;
    if (j > 0 && T[i * n + j - 1] < INFINITY) {
        const double v = node_r(E, i, j - 1) * T[i * n + j - 1];
        hx = 1; tqx = v; ux = T[i * n + j - 1]; sgx = 1.0;
    }
    if (j < n - 1 && T[i * n + j + 1] < INFINITY) {
        const double v = node_r(E, i, j + 1) * T[i * n + j + 1];
        if (!hx || v < tqx) { hx = 1; tqx = v; ux = T[i * n + j + 1]; sgx = -1.0; }
    }
    if (i > 0 && T[(i - 1) * n + j] < INFINITY) {
        const double v = node_r(E, i - 1, j) * T[(i - 1) * n + j];
        hy = 1; tqy = v; uy = T[(i - 1) * n + j]; sgy = 1.0;
    }
    if (i < ny - 1 && T[(i + 1) * n + j] < INFINITY) {
        const double v = node_r(E, i + 1, j) * T[(i + 1) * n + j];
        if (!hy || v < tqy) { hy = 1; tqy = v; uy = T[(i + 1) * n + j]; sgy = -1.0; }
    }
    double best = INFINITY, t;
    const double s2 = sp * sp;
    /* discrete d tau/dx = ax t - bx and d tau/dy = ay t - by */
    const double ax = sgx * r / h + gx, bx = sgx * r * ux / h;
    const double ay = sgy * r / h + gy, by = sgy * r * uy / h;
    if (hx && hy) {
        const double A = ax * ax + ay * ay, B = ax * bx + ay * by, C = (bx * bx + by * by) - s2;
        if (big_root(A, B, C, &t) && sgx * (ax * t - bx) >= 0.0 && sgy * (ay * t - by) >= 0.0 && t < best) best = t;
    }
    if (hx && sgx * ax > 0.0) {
        t = (bx + sgx * sp) / ax;
        if (t < best) best = t;
    }
    if (hy && sgy * ay > 0.0) {
        t = (by + sgy * sp) / ay;
        if (t < best) best = t;
    }
    return best;
}

/* Fixed nodes (within sqrt(2) h of the source) and +inf elsewhere; fixed[] may be NULL. */
static void init_field(const eik_t *E, double *T, unsigned char *fixed) {
    const int64_t n = E->nx, ny = E->ny;
    int64_t in = (int64_t)floor(E->ys / E->h + 0.5), jn = (int64_t)floor(E->xs / E->h + 0.5);
    if (in < 0) in = 0;
    if (in > ny - 1) in = ny - 1;
    if (jn < 0) jn = 0;
    if (jn > n - 1) jn = n - 1;
    const double ssrc = E->s[in * n + jn];
    const double rfix = sqrt(2.0) * E->h;
    for (int64_t i = 0; i < ny; ++i)
        for (int64_t j = 0; j < n; ++j) {
            const int f = node_r(E, i, j) <= rfix;
            T[i * n + j] = f ? (E->s[i * n + j] + ssrc) / 2.0 : INFINITY;
            if (fixed) fixed[i * n + j] = (unsigned char)f;
        }
}

static int check(int64_t nx, int64_t ny, double h, const double *s, double xs, double ys) {
    if (nx < 2 || ny < 2 || !(h > 0.0) || !s) return -1;
    if (!(xs >= 0.0 && xs <= (double)(nx - 1) * h && ys >= 0.0 && ys <= (double)(ny - 1) * h)) return -1;
    return 0;
}

int oracle_eik_sweep(int64_t n, int64_t ny, double h, const double *s, double xs, double ys, int32_t max_rounds,
                     double tol, double *tau1, int32_t *rounds, double *change) {
    if (check(n, ny, h, s, xs, ys) || !tau1 || max_rounds < 0) return -1;
    eik_t E = {n, ny, h, xs, ys, s};
    unsigned char *fixed = (unsigned char *)malloc((size_t)(n * ny));
    if (!fixed) return -2;
    init_field(&E, tau1, fixed);
    int32_t done = 0;
    double last = INFINITY;
    while (done < max_rounds) {
        double dmax = 0.0;
        for (int pass = 0; pass < 4; ++pass) {
            const int iup = pass < 2, jup = (pass % 2) == 0;
            for (int64_t a = 0; a < ny; ++a) {
                const int64_t i = iup ? a : ny - 1 - a;
                for (int64_t b = 0; b < n; ++b) {
                    const int64_t j = jup ? b : n - 1 - b;
                    if (fixed[i * n + j]) continue;
                    const double t = local_update(&E, tau1, i, j);
                    const double old = tau1[i * n + j];
                    if (t < old) {
                        const double d = old == INFINITY ? INFINITY : old - t;
                        if (d > dmax) dmax = d;
                        tau1[i * n + j] = t;
                    }
                }
            }
        }
        ++done;
        last = dmax;
        if (tol >= 0.0 && dmax <= tol) break;
    }
    if (rounds) *rounds = done;
    if (change) *change = last;
    free(fixed);
    return 0;
}
