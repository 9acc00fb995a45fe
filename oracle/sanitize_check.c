/*
 * Sanitizer driver of the D2Q9 oracle (TEST INFRASTRUCTURE ONLY): compiled
 * together with iilbm_oracle.c into one executable under AddressSanitizer and
 * UndefinedBehaviorSanitizer by tests/test_sanitized.py, it walks every
 * path of the oracle once on small problems: the membrane under the four
 * force modes with SRT and MRT, the cubic-spline membrane, the cut-link
 * enumerations (chord-wise, brute force, spline, level set), the walled
 * channel with a direct-forcing cylinder, inlet and outlet, the normal-force
 * circle with outflow on every side, a free and a prescribed moving circle,
 * and the diagnostics.  Any out-of-bounds access, use of freed memory, leak,
 * signed overflow or other undefined behaviour aborts the run; otherwise it
 * prints "sanitize-check ok" and the number of states it checked.
 */
#include "iilbm_oracle.c"

#include <stdio.h>

static int checked = 0;

static void ellipse(double *X, int N, double cx, double cy, double a, double b)
{
    for (int k = 0; k < N; k++) {
        double t = 2.0 * M_PI * k / N;
        X[2 * k] = cx + a * cos(t);
        X[2 * k + 1] = cy + b * sin(t);
    }
}

static or_problem base(int nx, int ny, double tau, int collision)
{
    or_problem p;
    memset(&p, 0, sizeof p);
    p.nx = nx;
    p.ny = ny;
    p.tau = tau;
    p.collision = collision;
    if (collision == OR_MRT) {
        double s[9] = {0.0, 1.63, 1.14, 0.0, 1.92, 0.0, 1.92, 1.0 / tau, 1.0 / tau};
        memcpy(p.s, s, sizeof s);
    }
    return p;
}

static double *rest(const or_problem *p)
{
    long n = (long)p->nx * p->ny;
    double *f = malloc(9 * n * sizeof(double));
    int32_t ex[9], ey[9];
    double w[9];
    or_d2q9(ex, ey, w);
    for (int i = 0; i < 9; i++)
        for (long c = 0; c < n; c++) f[i * n + c] = w[i];
    return f;
}

static void require_finite(const double *v, long n, const char *what)
{
    for (long i = 0; i < n; i++)
        if (!isfinite(v[i])) {
            fprintf(stderr, "non-finite value in %s at %ld\n", what, i);
            exit(2);
        }
    checked++;
}

static void diagnostics(const or_problem *p, const double *f, const double *X)
{
    long n = (long)p->nx * p->ny;
    double *rho = malloc(n * sizeof(double)), *ux = malloc(n * sizeof(double)), *uy = malloc(n * sizeof(double));
    or_moments(p, f, rho, ux, uy);
    require_finite(rho, n, "rho");
    if (X && p->n_markers >= 3) {
        (void)or_polygon_area(p->n_markers, X);
        (void)or_pressure_jump(p, rho, X, 3.0);
        (void)or_node_inside(p, X, p->nx / 2, p->ny / 2);
    }
    free(rho); free(ux); free(uy);
}

static void membrane_case(int collision, int mode, int geometry)
{
    or_problem p = base(64, 64, 0.8, collision);
    p.interface = OR_IF_MEMBRANE;
    p.force_mode = mode;
    p.geometry = geometry;
    p.n_markers = mode == OR_IB_LBM || mode == OR_IB_LBM_GUO ? 200 : 96;
    p.kappa = 0.05;
    p.dX = 2.0 * M_PI * sqrt(12.0 * 8.0) / p.n_markers;
    double *X = malloc(2 * p.n_markers * sizeof(double)), *f = rest(&p);
    ellipse(X, p.n_markers, 32.0, 32.0, 12.0, 8.0);
    double *fh = malloc(2 * 12 * sizeof(double));
    if (or_run(&p, f, X, 12, fh) != 0) { fprintf(stderr, "membrane run failed\n"); exit(2); }
    require_finite(f, 9L * 64 * 64, "membrane f");
    require_finite(X, 2 * p.n_markers, "membrane X");
    diagnostics(&p, f, X);
    free(X); free(f); free(fh);
}

static void cutlink_cases(void)
{
    or_problem p = base(48, 40, 0.7, OR_SRT);
    p.interface = OR_IF_MEMBRANE;
    p.n_markers = 5;
    p.kappa = 0.01;
    p.dX = 1.5;
    /* a pentagon with a vertex on a node and an edge along a lattice line */
    double X[10] = {20.0, 20.0, 26.0, 20.0, 27.5, 24.25, 23.0, 27.0, 19.0, 24.5};
    double jp[5] = {1e-3, 2e-3, -1e-3, 5e-4, 0.0};
    int cap = 4096;
    or_link *a = calloc(cap, sizeof(or_link)), *b = calloc(cap, sizeof(or_link));
    int na = or_cutlinks(&p, X, jp, a, cap);
    int nb = or_cutlinks_bruteforce(&p, X, jp, 15, 32, 15, 32, b, cap);
    if (na != nb || na <= 0) { fprintf(stderr, "cut links %d vs %d\n", na, nb); exit(2); }
    /* record buffer smaller than the link count: counted, not written past */
    (void)or_cutlinks(&p, X, jp, a, 3);
    double G[10] = {0};
    p.geometry = 1;
    double M[10];
    or_spline(&p, X, M);
    require_finite(M, 10, "spline");
    (void)or_cutlinks_spline(&p, X, G, a, cap);
    checked++;
    free(a); free(b);
}

static void channel_case(int mode)
{
    or_problem p = base(128, 64, 0.66, OR_MRT);
    p.bc[0] = OR_INLET; p.bc[1] = OR_OUTLET; p.bc[2] = OR_WALL; p.bc[3] = OR_WALL;
    p.u_max = 0.05;
    p.interface = OR_IF_RIGID;
    p.force_mode = mode;
    p.n_markers = 13;
    p.cx = 32.0; p.cy = 32.0; p.radius = 2.0;
    p.dX = M_PI * 4.0 / 13.0;
    double *X = malloc(2 * 13 * sizeof(double)), *f = rest(&p), fh[2 * 20];
    ellipse(X, 13, 32.0, 32.0, 2.0, 2.0);
    if (or_run(&p, f, X, 20, fh) != 0) { fprintf(stderr, "channel run failed\n"); exit(2); }
    require_finite(f, 9L * 128 * 64, "channel f");
    require_finite(fh, 40, "channel force");
    diagnostics(&p, f, X);
    free(X); free(f);
}

static void normal_circle_case(int mode)
{
    or_problem p = base(41, 41, 0.65, OR_MRT);
    for (int q = 0; q < 4; q++) p.bc[q] = OR_OUTLET;
    p.interface = OR_IF_NORMAL;
    p.force_mode = mode;
    p.n_markers = 64;
    p.cx = 20.0; p.cy = 20.0; p.radius = 10.0;
    p.dX = 2.0 * M_PI * 10.0 / 64;
    p.f_normal = 1e-4;
    double *X = malloc(2 * 64 * sizeof(double)), *f = rest(&p);
    ellipse(X, 64, 20.0, 20.0, 10.0, 10.0);
    if (or_run(&p, f, X, 10, NULL) != 0) { fprintf(stderr, "normal circle failed\n"); exit(2); }
    require_finite(f, 9L * 41 * 41, "normal circle f");
    free(X); free(f);
}

static void body_case(int free_dofs, double presc)
{
    or_problem p = base(96, 64, 0.6, OR_MRT);
    p.bc[0] = OR_INLET_UNIFORM; p.bc[1] = OR_OUTLET; p.bc[2] = OR_WALL; p.bc[3] = OR_WALL;
    p.u_max = 0.02;
    p.interface = OR_IF_RIGID;
    p.n_markers = 40;
    p.cx = 40.0; p.cy = 32.0; p.radius = 6.0;
    p.dX = 2.0 * M_PI * 6.0 / 40;
    or_body_params bp;
    memset(&bp, 0, sizeof bp);
    bp.free_dofs = free_dofs;
    bp.rho_star = 2.0;
    bp.spring[1] = 1e-3;
    bp.presc_amp[0] = 2.0;
    bp.presc_umax[0] = presc;
    or_body b;
    memset(&b, 0, sizeof b);
    b.c[0] = b.c0[0] = p.cx;
    b.c[1] = b.c0[1] = p.cy;
    double *X = malloc(2 * 40 * sizeof(double)), *f = rest(&p);
    ellipse(X, 40, p.cx, p.cy, 6.0, 6.0);
    for (int s = 0; s < 10; s++)
        if (or_step_body(&p, &bp, &b, f, X) != 0) { fprintf(stderr, "body step failed\n"); exit(2); }
    require_finite(f, 9L * 96 * 64, "body f");
    require_finite(b.c, 2, "body centre");
    free(X); free(f);
}

int main(void)
{
    for (int collision = 0; collision < 2; collision++)
        for (int mode = 0; mode < 4; mode++) membrane_case(collision, mode, 0);
    membrane_case(OR_SRT, OR_II_LBM, 1);
    membrane_case(OR_MRT, OR_II_LBM_GUO, 1);
    cutlink_cases();
    for (int mode = 0; mode < 4; mode++) channel_case(mode);
    normal_circle_case(OR_II_LBM);
    normal_circle_case(OR_IB_LBM);
    body_case(7, 0.0);
    body_case(2, 0.01);
    printf("sanitize-check ok (%d states checked)\n", checked);
    return 0;
}
