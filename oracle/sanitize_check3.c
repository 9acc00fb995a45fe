/*
 * Sanitizer driver of the D3Q19 oracle (TEST INFRASTRUCTURE ONLY): compiled
 * together with iilbm3_oracle.c into one executable under AddressSanitizer and
 * UndefinedBehaviorSanitizer by tests/test_sanitized.py.  It walks the
 * level-set sphere (II-LBM and IB-LBM, SRT and MRT), the fixed triangulated
 * surface, the deformable membrane under II-LBM and IB-LBM, the rigid surface
 * and the free sphere once each, on a small periodic box with a geodesic
 * sphere built here (an octahedron split three times, 512 triangles).
 */
#include "iilbm3_oracle.c"

#include <stdio.h>

static int checked = 0;

/* geodesic sphere: vertices X[3 nv], triangles tri[3 nt], counter-clockwise
 * seen from outside */
static int nv_, nt_;
static double Xs[3 * 2048];
static int32_t Ts[3 * 4096];

static int midpoint(int a, int b)
{
    double m[3];
    for (int k = 0; k < 3; k++) m[k] = 0.5 * (Xs[3 * a + k] + Xs[3 * b + k]);
    for (int v = 0; v < nv_; v++)
        if (fabs(Xs[3 * v] - m[0]) + fabs(Xs[3 * v + 1] - m[1]) + fabs(Xs[3 * v + 2] - m[2]) < 1e-12)
            return v;
    memcpy(Xs + 3 * nv_, m, sizeof m);
    return nv_++;
}

static void geodesic(double cx, double cy, double cz, double R)
{
    const double oct[6][3] = {{1, 0, 0}, {-1, 0, 0}, {0, 1, 0}, {0, -1, 0}, {0, 0, 1}, {0, 0, -1}};
    const int faces[8][3] = {{0, 2, 4}, {2, 1, 4}, {1, 3, 4}, {3, 0, 4},
                             {2, 0, 5}, {1, 2, 5}, {3, 1, 5}, {0, 3, 5}};
    nv_ = 6;
    nt_ = 8;
    memcpy(Xs, oct, sizeof oct);
    memcpy(Ts, faces, sizeof faces);
    for (int level = 0; level < 3; level++) {
        int32_t T2[3 * 4096];
        int n2 = 0;
        for (int t = 0; t < nt_; t++) {
            int a = Ts[3 * t], b = Ts[3 * t + 1], c = Ts[3 * t + 2];
            int ab = midpoint(a, b), bc = midpoint(b, c), ca = midpoint(c, a);
            int q[4][3] = {{a, ab, ca}, {ab, b, bc}, {ca, bc, c}, {ab, bc, ca}};
            for (int s = 0; s < 4; s++)
                for (int k = 0; k < 3; k++) T2[3 * n2 + 3 * s + k] = q[s][k];
            n2 += 4;
        }
        memcpy(Ts, T2, sizeof(int32_t) * 3 * n2);
        nt_ = n2;
    }
    for (int v = 0; v < nv_; v++) {
        double *x = Xs + 3 * v, r = sqrt(x[0] * x[0] + x[1] * x[1] + x[2] * x[2]);
        x[0] = cx + R * x[0] / r;
        x[1] = cy + R * x[1] / r;
        x[2] = cz + R * x[2] / r;
    }
}

static or3_problem box(int n, int collision, int mode)
{
    or3_problem p;
    memset(&p, 0, sizeof p);
    p.nx = p.ny = p.nz = n;
    p.force_mode = mode;
    p.tau = 0.8;
    p.collision = collision;
    for (int k = 0; k < 19; k++) p.s[k] = 1.0 / p.tau;
    p.s[0] = p.s[3] = p.s[5] = p.s[7] = 0.0;
    p.s[1] = 1.19;
    p.s[2] = 1.4;
    return p;
}

static double *rest(const or3_problem *p)
{
    long n = (long)p->nx * p->ny * p->nz;
    double *f = malloc((size_t)Q * n * sizeof(double));
    for (int i = 0; i < Q; i++)
        for (long c = 0; c < n; c++) f[i * n + c] = wt3(i);
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

int main(void)
{
    const int n = 20;
    const long cells = (long)n * n * n;
    for (int collision = 0; collision < 2; collision++)
        for (int mode = 0; mode < 2; mode++) {
            or3_problem p = box(n, collision, mode);
            p.cx = 10.2; p.cy = 9.7; p.cz = 10.4; p.radius = 5.0;
            p.f_normal = 1e-4;
            p.n_markers = 320;
            double *f = rest(&p), *X = malloc(sizeof(double) * 3 * p.n_markers);
            for (int k = 0; k < p.n_markers; k++) {   /* Fibonacci points on the sphere */
                double z = 1.0 - (2.0 * k + 1.0) / p.n_markers, r = sqrt(1.0 - z * z);
                double ph = k * M_PI * (3.0 - sqrt(5.0));
                X[3 * k] = p.cx + p.radius * r * cos(ph);
                X[3 * k + 1] = p.cy + p.radius * r * sin(ph);
                X[3 * k + 2] = p.cz + p.radius * z;
            }
            if (or3_run(&p, f, X, 5) != 0) { fprintf(stderr, "sphere run failed\n"); return 2; }
            require_finite(f, Q * cells, "sphere f");
            (void)or3_count_cut_links(&p);
            free(f); free(X);
        }
    geodesic(10.13, 9.71, 10.37, 5.0);
    {
        or3_problem p = box(n, 0, 0);
        double *f = rest(&p), *pv = malloc(sizeof(double) * nv_);
        for (int v = 0; v < nv_; v++) pv[v] = 1e-4 * (1.0 + 0.1 * (v % 3));
        if (or3_run_mesh(&p, f, nv_, Xs, nt_, Ts, pv, 5) != 0) { fprintf(stderr, "mesh run failed\n"); return 2; }
        require_finite(f, Q * cells, "mesh f");
        free(f); free(pv);
    }
    for (int law = 0; law < 3; law++)
        for (int collision = 0; collision < 2; collision++) {
            or3_problem p = box(n, collision, 0);
            double *f = rest(&p), *X = malloc(sizeof(double) * 3 * nv_), U[3 * 2048], F[3];
            memcpy(X, Xs, sizeof(double) * 3 * nv_);
            for (int v = 0; v < nv_; v++) X[3 * v] = 10.13 + 1.2 * (X[3 * v] - 10.13);   /* stretched */
            if (law == 1) { p.body[0] = 1e-6; }
            if (or3_run_surface(&p, f, nv_, X, nt_, Ts, law, 0.01, 5, U, F) != 0) {
                fprintf(stderr, "surface law %d failed\n", law);
                return 2;
            }
            require_finite(f, Q * cells, "surface f");
            require_finite(X, 3 * nv_, "surface X");
            free(f); free(X);
        }
    {
        or3_problem p = box(n, 0, 0);
        p.body[0] = 1e-6;
        double *f = rest(&p), *X = malloc(sizeof(double) * 3 * nv_), body[21] = {0}, F[3], T[3];
        memcpy(X, Xs, sizeof(double) * 3 * nv_);
        body[0] = 10.13; body[1] = 9.71; body[2] = 10.37;
        if (or3_run_free_sphere(&p, f, nv_, X, nt_, Ts, 5.0, 1.5, body, 5, F, T) != 0) {
            fprintf(stderr, "free sphere failed\n");
            return 2;
        }
        require_finite(body, 21, "free sphere state");
        free(f); free(X);
    }
    printf("sanitize-check3 ok (%d states checked)\n", checked);
    return 0;
}
