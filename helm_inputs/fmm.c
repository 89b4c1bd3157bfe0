/*
 * First-order fast-marching solver for the eikonal equation |grad T| = s(x)
 * on a uniform grid of nx columns and ny rows of nodes with spacing h (Sethian's upwind
 * scheme).
 *
 * The phase field that demodulates the level-2 residual is the first-arrival
 * travel time from the source(s) (the paper's eikonal equation for the phase,
 * Section 3.2).  This file only builds that INPUT field; it holds none of the
 * solver's arithmetic.
 *
 * Layout: row-major, index i*nx + j with i the y index and j the x index.
 * Seeds: for every source, the 5x5 box of nodes around the node nearest x0 is
 * set to s(x0_node) * |x - x0| (minimum over sources) and frozen.
 * Heap ties are broken by (value, linear index), which makes the result
 * independent of insertion order.
 *
 * Returns 0 on success, -1 on bad arguments, -2 on allocation failure.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>

typedef struct {
    double *key;
    int64_t *node;
    int64_t *pos; /* pos[node] = heap slot or -1 */
    int64_t size;
} heap_t;

static int less(const heap_t *H, int64_t a, int64_t b) {
    if (H->key[a] < H->key[b]) return 1;
    if (H->key[a] > H->key[b]) return 0;
    return H->node[a] < H->node[b];
}

static void swap_slots(heap_t *H, int64_t a, int64_t b) {
    double tk = H->key[a];
    int64_t tn = H->node[a];
    H->key[a] = H->key[b];
    H->node[a] = H->node[b];
    H->key[b] = tk;
    H->node[b] = tn;
    H->pos[H->node[a]] = a;
    H->pos[H->node[b]] = b;
}

static void sift_up(heap_t *H, int64_t s) {
    while (s > 0) {
        int64_t p = (s - 1) / 2;
        if (!less(H, s, p)) break;
        swap_slots(H, s, p);
        s = p;
    }
}

static void sift_down(heap_t *H, int64_t s) {
    for (;;) {
        int64_t l = 2 * s + 1, r = l + 1, m = s;
        if (l < H->size && less(H, l, m)) m = l;
        if (r < H->size && less(H, r, m)) m = r;
        if (m == s) break;
        swap_slots(H, s, m);
        s = m;
    }
}

static void heap_push_or_decrease(heap_t *H, int64_t node, double key) {
    int64_t p = H->pos[node];
    if (p < 0) {
        p = H->size++;
        H->key[p] = key;
        H->node[p] = node;
        H->pos[node] = p;
        sift_up(H, p);
    } else if (key < H->key[p]) {
        H->key[p] = key;
        sift_up(H, p);
    }
}

static int64_t heap_pop(heap_t *H) {
    int64_t top = H->node[0];
    H->pos[top] = -1;
    H->size--;
    if (H->size > 0) {
        H->key[0] = H->key[H->size];
        H->node[0] = H->node[H->size];
        H->pos[H->node[0]] = 0;
        sift_down(H, 0);
    }
    return top;
}

/* Upwind update at (i,j) from frozen neighbours. */
static double local_update(const double *T, const unsigned char *frozen, int64_t nx, int64_t ny,
                           int64_t i, int64_t j, double hs) {
    double a = INFINITY, b = INFINITY;
    if (i > 0 && frozen[(i - 1) * nx + j]) a = T[(i - 1) * nx + j];
    if (i + 1 < ny && frozen[(i + 1) * nx + j] && T[(i + 1) * nx + j] < a) a = T[(i + 1) * nx + j];
    if (j > 0 && frozen[i * nx + j - 1]) b = T[i * nx + j - 1];
    if (j + 1 < nx && frozen[i * nx + j + 1] && T[i * nx + j + 1] < b) b = T[i * nx + j + 1];
    double lo = a < b ? a : b, hi = a < b ? b : a;
    if (!isfinite(lo)) return INFINITY;
    if (!isfinite(hi) || hi - lo >= hs) return lo + hs;
    /* (T-a)^2 + (T-b)^2 = hs^2 */
    double d = hi - lo;
    return 0.5 * (lo + hi + sqrt(2.0 * hs * hs - d * d));
}

int fmm_eikonal(int64_t nx, int64_t ny, double h, const double *slowness, int64_t nsrc,
                const double *src_xy, double *T) {
    if (nx < 4 || ny < 4 || h <= 0 || nsrc < 1 || !slowness || !src_xy || !T) return -1;
    int64_t N = nx * ny;
    unsigned char *frozen = (unsigned char *)calloc((size_t)N, 1);
    heap_t H;
    H.key = (double *)malloc((size_t)N * sizeof(double));
    H.node = (int64_t *)malloc((size_t)N * sizeof(int64_t));
    H.pos = (int64_t *)malloc((size_t)N * sizeof(int64_t));
    H.size = 0;
    if (!frozen || !H.key || !H.node || !H.pos) {
        free(frozen); free(H.key); free(H.node); free(H.pos);
        return -2;
    }
    for (int64_t p = 0; p < N; ++p) { T[p] = INFINITY; H.pos[p] = -1; }

    for (int64_t s = 0; s < nsrc; ++s) {
        double x0 = src_xy[2 * s], y0 = src_xy[2 * s + 1];
        int64_t jc = (int64_t)llround(x0 / h), ic = (int64_t)llround(y0 / h);
        if (jc < 0) jc = 0;
        if (jc > nx - 1) jc = nx - 1;
        if (ic < 0) ic = 0;
        if (ic > ny - 1) ic = ny - 1;
        double s0 = slowness[ic * nx + jc];
        for (int64_t di = -2; di <= 2; ++di)
            for (int64_t dj = -2; dj <= 2; ++dj) {
                int64_t i = ic + di, j = jc + dj;
                if (i < 0 || j < 0 || i >= ny || j >= nx) continue;
                double dx = j * h - x0, dy = i * h - y0;
                double t = s0 * sqrt(dx * dx + dy * dy);
                if (t < T[i * nx + j]) T[i * nx + j] = t;
                frozen[i * nx + j] = 1;
            }
    }
    /* initial trial band */
    for (int64_t p = 0; p < N; ++p) {
        if (!frozen[p]) continue;
        int64_t i = p / nx, j = p % nx;
        const int64_t nb[4][2] = {{i - 1, j}, {i + 1, j}, {i, j - 1}, {i, j + 1}};
        for (int q = 0; q < 4; ++q) {
            int64_t a = nb[q][0], b = nb[q][1];
            if (a < 0 || b < 0 || a >= ny || b >= nx || frozen[a * nx + b]) continue;
            double t = local_update(T, frozen, nx, ny, a, b, h * slowness[a * nx + b]);
            if (t < T[a * nx + b]) T[a * nx + b] = t;
            heap_push_or_decrease(&H, a * nx + b, T[a * nx + b]);
        }
    }
    while (H.size > 0) {
        int64_t p = heap_pop(&H);
        frozen[p] = 1;
        int64_t i = p / nx, j = p % nx;
        const int64_t nb[4][2] = {{i - 1, j}, {i + 1, j}, {i, j - 1}, {i, j + 1}};
        for (int q = 0; q < 4; ++q) {
            int64_t a = nb[q][0], b = nb[q][1];
            if (a < 0 || b < 0 || a >= ny || b >= nx || frozen[a * nx + b]) continue;
            double t = local_update(T, frozen, nx, ny, a, b, h * slowness[a * nx + b]);
            if (t < T[a * nx + b]) {
                T[a * nx + b] = t;
                heap_push_or_decrease(&H, a * nx + b, t);
            }
        }
    }
    free(frozen); free(H.key); free(H.node); free(H.pos);
    return 0;
}
