/*
 * oracle.c -- plain FP64 CPU reference for iterated Jacobi stencil sweeps.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark use it.  It shares no code, header, table or helper
 * with the GPU path.
 *
 * What it computes (the definition, not an optimisation of it):
 *
 *   Section 1 (Introduction) of the paper defines a stencil of order r as an
 *   update in which a point at the next time step is a weighted sum of the
 *   (2r+1) points per direction around it at the previous step, and the naive
 *   implementation of a d-dimensional stencil as d+1 nested loops with time
 *   outermost.  Section 2.1 (the 1D3P example) and Section 3.3 (last
 *   paragraph) fix the Jacobi semantics: two arrays, one holding time t and
 *   one holding time t+1.
 *
 *   For t = 0..T-1 and every grid point x:
 *       u_{t+1}[x] = sum_j c_j * g(u_t, x + o_j)        (j in canonical order)
 *   with g(u, y) = u[y] inside the grid, 0 outside (zero halo), or
 *   u[y mod N] per axis (periodic).
 *
 * Readings taken where the paper is silent:
 *   - offset sets: star = {0} U {+-j e_i : 1<=j<=r}, box = {o : max|o_i| <= r};
 *   - canonical coefficient order: offsets sorted lexicographically with
 *     axis 0 (the slowest, row-major) most significant, each component
 *     ascending from -r to +r;
 *   - layout: row-major, axis d-1 unit stride;
 *   - boundary: zero halo of width r held at 0 at every step, or periodic;
 *   - arithmetic: each product rounded, products summed left to right in
 *     canonical order, no FMA contraction (built with -ffp-contract=off).
 *
 * The adjoint (reverse-mode derivative of the sweep) is not in the paper; it
 * follows from the definition above: with lambda_T = dL/du_T,
 *       lambda_t[z] = sum_j c_j * g(lambda_{t+1}, z - o_j)
 *       dL/dc_j    += sum_x lambda_{t+1}[x] * g(u_t, x + o_j)
 * and dL/du_0 = lambda_0.  The forward states u_t are recovered from stored
 * checkpoints every `ckpt` steps by re-running the forward loop.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <time.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORACLE_STAR 0
#define ORACLE_BOX 1
#define ORACLE_BC_ZERO 0
#define ORACLE_BC_PERIODIC 1

/* Number of points of a d-dimensional star or box stencil of order r. */
int oracle_num_points(int dim, int r, int kind)
{
    if (dim < 1 || dim > 3 || r < 1 || (kind != ORACLE_STAR && kind != ORACLE_BOX))
        return -1;
    if (kind == ORACLE_STAR)
        return 2 * dim * r + 1;
    int n = 1;
    for (int i = 0; i < dim; ++i)
        n *= 2 * r + 1;
    return n;
}

/*
 * Enumerate the offset set in canonical order: walk every tuple of
 * [-r, r]^dim lexicographically (axis 0 slowest) and keep the members of the
 * set.  A star keeps tuples with at most one non-zero component.
 * out receives npts*dim ints; returns npts, or -1 on bad arguments.
 */
int oracle_offsets(int dim, int r, int kind, int32_t *out)
{
    int npts = oracle_num_points(dim, r, kind);
    if (npts < 0 || out == NULL)
        return -1;
    int side = 2 * r + 1;
    int total = 1;
    for (int i = 0; i < dim; ++i)
        total *= side;
    int n = 0;
    for (int code = 0; code < total; ++code) {
        int o[3];
        int rest = code;
        for (int i = dim - 1; i >= 0; --i) { /* last axis varies fastest */
            o[i] = rest % side - r;
            rest /= side;
        }
        int nonzero = 0;
        for (int i = 0; i < dim; ++i)
            nonzero += (o[i] != 0);
        if (kind == ORACLE_STAR && nonzero > 1)
            continue;
        for (int i = 0; i < dim; ++i)
            out[n * dim + i] = o[i];
        ++n;
    }
    return n;
}

/* Per-axis view of a grid padded to three axes (missing leading axes have
 * extent 1 and offset 0, so they never leave the grid). */
typedef struct {
    int64_t n[3];
    int npts;
    int32_t off[729 * 3]; /* r <= 4 box in 3D has 9^3 = 729 points */
    double c[729];
    int bc;
} grid3;

static int make_grid3(grid3 *g, int dim, const int64_t *shape, int r, int kind,
                      const double *coef, int bc, int sign)
{
    if (dim < 1 || dim > 3 || r < 1 || r > 4 || shape == NULL || coef == NULL)
        return -1;
    if (bc != ORACLE_BC_ZERO && bc != ORACLE_BC_PERIODIC)
        return -1;
    int32_t tmp[729 * 3];
    int npts = oracle_offsets(dim, r, kind, tmp);
    if (npts < 0)
        return -1;
    for (int i = 0; i < 3; ++i)
        g->n[i] = 1;
    for (int i = 0; i < dim; ++i) {
        if (shape[i] < 1)
            return -1;
        g->n[3 - dim + i] = shape[i];
    }
    g->npts = npts;
    g->bc = bc;
    for (int j = 0; j < npts; ++j) {
        for (int i = 0; i < 3; ++i)
            g->off[j * 3 + i] = 0;
        for (int i = 0; i < dim; ++i)
            g->off[j * 3 + 3 - dim + i] = sign * tmp[j * dim + i];
        g->c[j] = coef[j];
    }
    return 0;
}

/* g(u, y): the grid value at coordinate y, with the boundary rule applied. */
static double fetch(const grid3 *g, const double *u, int64_t y0, int64_t y1, int64_t y2)
{
    int64_t y[3] = {y0, y1, y2};
    for (int i = 0; i < 3; ++i) {
        if (y[i] < 0 || y[i] >= g->n[i]) {
            if (g->bc == ORACLE_BC_ZERO)
                return 0.0;
            y[i] = ((y[i] % g->n[i]) + g->n[i]) % g->n[i];
        }
    }
    return u[(y[0] * g->n[1] + y[1]) * g->n[2] + y[2]];
}

/* One Jacobi step: dst[x] = sum_j c_j * g(src, x + off_j). */
static void sweep_once(const grid3 *g, const double *src, double *dst)
{
    const int64_t n0 = g->n[0], n1 = g->n[1], n2 = g->n[2];
#pragma omp parallel for collapse(3) schedule(static)
    for (int64_t x0 = 0; x0 < n0; ++x0)
        for (int64_t x1 = 0; x1 < n1; ++x1)
            for (int64_t x2 = 0; x2 < n2; ++x2) {
                double acc = 0.0;
                for (int j = 0; j < g->npts; ++j) {
                    double v = fetch(g, src, x0 + g->off[3 * j], x1 + g->off[3 * j + 1],
                                     x2 + g->off[3 * j + 2]);
                    acc += g->c[j] * v;
                }
                dst[(x0 * n1 + x1) * n2 + x2] = acc;
            }
}

static void set_threads(int nthreads)
{
#ifdef _OPENMP
    if (nthreads > 0)
        omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
}

int oracle_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/*
 * T Jacobi steps from u0 into uT (both hold prod(shape) doubles, row-major).
 * u0 and uT may be the same array.  nthreads <= 0 keeps the OpenMP default.
 * If seconds != NULL it receives the CLOCK_MONOTONIC time of the time loop.
 * Returns 0, or -1 on bad arguments, -3 on allocation failure.
 */
int oracle_run(int dim, const int64_t *shape, int r, int kind, const double *coef, int bc,
               int64_t T, const double *u0, double *uT, int nthreads, double *seconds)
{
    grid3 g;
    if (make_grid3(&g, dim, shape, r, kind, coef, bc, +1) != 0 || T < 0 || !u0 || !uT)
        return -1;
    set_threads(nthreads);
    int64_t n = g.n[0] * g.n[1] * g.n[2];
    double *a = (double *)malloc((size_t)n * sizeof(double));
    double *b = (double *)malloc((size_t)n * sizeof(double));
    if (!a || !b) {
        free(a);
        free(b);
        return -3;
    }
    memcpy(a, u0, (size_t)n * sizeof(double));
    struct timespec t0, t1;
    clock_gettime(CLOCK_MONOTONIC, &t0);
    for (int64_t t = 0; t < T; ++t) { /* time outermost */
        sweep_once(&g, a, b);
        double *s = a;
        a = b;
        b = s;
    }
    clock_gettime(CLOCK_MONOTONIC, &t1);
    if (seconds)
        *seconds = (double)(t1.tv_sec - t0.tv_sec) + 1e-9 * (double)(t1.tv_nsec - t0.tv_nsec);
    memcpy(uT, a, (size_t)n * sizeof(double));
    free(a);
    free(b);
    return 0;
}

/*
 * Reverse-mode derivative of T steps.  gT = dL/du_T on entry; on return
 * grad_u0 = dL/du_0 and grad_c[j] = dL/dc_j (npts doubles, overwritten).
 * Forward states are rebuilt from checkpoints u_0, u_ckpt, u_2ckpt, ...:
 * each segment is re-run from its checkpoint with every state of the
 * segment kept, then walked backwards.
 */
int oracle_adjoint(int dim, const int64_t *shape, int r, int kind, const double *coef, int bc,
                   int64_t T, int64_t ckpt, const double *u0, const double *gT,
                   double *grad_u0, double *grad_c, int nthreads)
{
    grid3 fwd, adj;
    if (make_grid3(&fwd, dim, shape, r, kind, coef, bc, +1) != 0 ||
        make_grid3(&adj, dim, shape, r, kind, coef, bc, -1) != 0)
        return -1;
    if (T < 0 || ckpt < 1 || !u0 || !gT || !grad_u0 || !grad_c)
        return -1;
    set_threads(nthreads);
    const int64_t n = fwd.n[0] * fwd.n[1] * fwd.n[2];
    const int64_t nseg = T > 0 ? (T + ckpt - 1) / ckpt : 0;
    const int64_t seglen = T < ckpt ? T : ckpt;
    double *ck = (double *)malloc((size_t)(nseg > 0 ? nseg : 1) * n * sizeof(double));
    double *seg = (double *)malloc((size_t)(seglen + 1) * n * sizeof(double));
    double *lam = (double *)malloc((size_t)n * sizeof(double));
    double *tmp = (double *)malloc((size_t)n * sizeof(double));
    if (!ck || !seg || !lam || !tmp) {
        free(ck);
        free(seg);
        free(lam);
        free(tmp);
        return -3;
    }
    for (int j = 0; j < fwd.npts; ++j)
        grad_c[j] = 0.0;

    /* forward pass, keeping u_{s*ckpt} */
    memcpy(tmp, u0, (size_t)n * sizeof(double));
    for (int64_t t = 0; t < T; ++t) {
        if (t % ckpt == 0)
            memcpy(ck + (t / ckpt) * n, tmp, (size_t)n * sizeof(double));
        sweep_once(&fwd, tmp, lam);
        memcpy(tmp, lam, (size_t)n * sizeof(double));
    }

    memcpy(lam, gT, (size_t)n * sizeof(double));
    const int64_t n0 = fwd.n[0], n1 = fwd.n[1], n2 = fwd.n[2];
    for (int64_t s = nseg - 1; s >= 0; --s) {
        int64_t tb = s * ckpt;
        int64_t te = tb + ckpt < T ? tb + ckpt : T;
        /* seg[i] = u_{tb+i} for i = 0 .. te-tb-1 */
        memcpy(seg, ck + s * n, (size_t)n * sizeof(double));
        for (int64_t t = tb + 1; t < te; ++t)
            sweep_once(&fwd, seg + (t - 1 - tb) * n, seg + (t - tb) * n);
        for (int64_t t = te - 1; t >= tb; --t) {
            const double *ut = seg + (t - tb) * n;
            /* dL/dc_j += sum_x lambda_{t+1}[x] * g(u_t, x + o_j) */
            for (int j = 0; j < fwd.npts; ++j) {
                double acc = 0.0;
#pragma omp parallel for collapse(3) reduction(+ : acc) schedule(static)
                for (int64_t x0 = 0; x0 < n0; ++x0)
                    for (int64_t x1 = 0; x1 < n1; ++x1)
                        for (int64_t x2 = 0; x2 < n2; ++x2)
                            acc += lam[(x0 * n1 + x1) * n2 + x2] *
                                   fetch(&fwd, ut, x0 + fwd.off[3 * j], x1 + fwd.off[3 * j + 1],
                                         x2 + fwd.off[3 * j + 2]);
                grad_c[j] += acc;
            }
            /* lambda_t[z] = sum_j c_j * g(lambda_{t+1}, z - o_j) */
            sweep_once(&adj, lam, tmp);
            memcpy(lam, tmp, (size_t)n * sizeof(double));
        }
    }
    memcpy(grad_u0, lam, (size_t)n * sizeof(double));
    free(ck);
    free(seg);
    free(lam);
    free(tmp);
    return 0;
}
