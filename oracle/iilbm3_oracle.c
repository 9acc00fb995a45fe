/*
 * Plain FP64 CPU oracle of a D3Q19 immersed interface-lattice Boltzmann step
 * (the three-dimensional form the paper's conclusion calls straightforward;
 * reading R28): a periodic box, single- or multiple-relaxation-time collision
 * (reading R30) with the He-Luo equilibrium and the simple force term
 * (Sec. 2.2.1-2.2.2 written for nineteen velocities), and a fixed sphere
 * carrying a uniform normal force F
 * per unit area, entered either
 *   - II-LBM: through the jump [[f_i]] = sigma w_i [[p]] / c_s^2 with
 *     [[p]] = F on every link the sphere's level set cuts (Sec. 3.1,
 *     Eq. (32); Sec. 3.2, Eq. (47)), or
 *   - IB-LBM: spread from surface markers with the three-dimensional product of
 *     Peskin's four-point delta (Sec. 2.2.2, Eq. (17));
 * and the same jumps on the links that cross a fixed closed triangulated
 * surface with a pressure jump given at its vertices (reading R29, at the end
 * of this file).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may call, link or
 * load this file.  It shares no code, header, table or helper with the GPU
 * library.
 *
 * Lattice units, f[i][z][y][x] with x fastest; markers X[k][3].
 */
#define _GNU_SOURCE
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define Q 19
static const int EX3[Q] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0};
static const int EY3[Q] = {0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, 1, -1};
static const int EZ3[Q] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1};
static const double CS2 = 1.0 / 3.0;

static double wt3(int i)
{
    if (i == 0) return 1.0 / 3.0;
    if (i <= 6) return 1.0 / 18.0;
    return 1.0 / 36.0;
}

typedef struct {
    int32_t nx, ny, nz, force_mode;   /* 0 II-LBM, 1 IB-LBM */
    double tau;
    double cx, cy, cz, radius;         /* the sphere */
    double f_normal;                   /* F per unit area along the outward normal */
    int32_t n_markers;                 /* IB-LBM markers on the sphere */
    int32_t collision;                 /* 0 SRT, 1 MRT (reading R30) */
    double body[3];                    /* uniform body force */
    double s[19];                      /* MRT relaxation rates of the moments below */
} or3_problem;

static long id3(const or3_problem *p, int i, int x, int y, int z)
{
    return (((long)i * p->nz + z) * p->ny + y) * p->nx + x;
}

static int wrap(int v, int n) { return ((v % n) + n) % n; }

void or3_lattice(int *ex, int *ey, int *ez, double *w)
{
    for (int i = 0; i < Q; i++) { ex[i] = EX3[i]; ey[i] = EY3[i]; ez[i] = EZ3[i]; w[i] = wt3(i); }
}

/* He-Luo incompressible equilibrium, w_i [rho + e.u / c_s^2 + (e.u)^2 / (2 c_s^4)
 * - u.u / (2 c_s^2)] (Sec. 2.2.1 with nineteen velocities). */
void or3_equilibrium(double rho, double ux, double uy, double uz, double *feq)
{
    double uu = ux * ux + uy * uy + uz * uz;
    for (int i = 0; i < Q; i++) {
        double eu = EX3[i] * ux + EY3[i] * uy + EZ3[i] * uz;
        feq[i] = wt3(i) * (rho + eu / CS2 + eu * eu / (2.0 * CS2 * CS2) - uu / (2.0 * CS2));
    }
}

/* The orthogonal D3Q19 moment basis of d'Humieres et al. (2002), the 3-D
 * counterpart of the Lallemand-Luo basis the paper's MRT uses (Sec. 2.2.1;
 * reading R30), row k as a polynomial in e = (cx, cy, cz), c2 = |e|^2:
 *   0 rho: 1            1 e: 19 c2 - 30        2 eps: (21 c2^2 - 53 c2 + 24) / 2
 *   3 jx: cx            4 qx: (5 c2 - 9) cx    5 jy: cy       6 qy: (5 c2 - 9) cy
 *   7 jz: cz            8 qz: (5 c2 - 9) cz
 *   9 3pxx: 3 cx^2 - c2                     10 3pixx: (3 c2 - 5)(3 cx^2 - c2)
 *  11 pww: cy^2 - cz^2                      12 piww: (3 c2 - 5)(cy^2 - cz^2)
 *  13 pxy: cx cy   14 pyz: cy cz   15 pxz: cx cz
 *  16 mx: cx (cy^2 - cz^2)   17 my: cy (cz^2 - cx^2)   18 mz: cz (cx^2 - cy^2) */
static double basis3(int k, int cx, int cy, int cz)
{
    const double x = cx, y = cy, z = cz, c2 = x * x + y * y + z * z;
    switch (k) {
    case 0: return 1.0;
    case 1: return 19.0 * c2 - 30.0;
    case 2: return (21.0 * c2 * c2 - 53.0 * c2 + 24.0) / 2.0;
    case 3: return x;
    case 4: return (5.0 * c2 - 9.0) * x;
    case 5: return y;
    case 6: return (5.0 * c2 - 9.0) * y;
    case 7: return z;
    case 8: return (5.0 * c2 - 9.0) * z;
    case 9: return 3.0 * x * x - c2;
    case 10: return (3.0 * c2 - 5.0) * (3.0 * x * x - c2);
    case 11: return y * y - z * z;
    case 12: return (3.0 * c2 - 5.0) * (y * y - z * z);
    case 13: return x * y;
    case 14: return y * z;
    case 15: return x * z;
    case 16: return x * (y * y - z * z);
    case 17: return y * (z * z - x * x);
    default: return z * (x * x - y * y);
    }
}

void or3_basis(double *M)
{
    for (int k = 0; k < Q; k++)
        for (int i = 0; i < Q; i++) M[k * Q + i] = basis3(k, EX3[i], EY3[i], EZ3[i]);
}

void or3_moments(const or3_problem *p, const double *f, double *rho, double *ux, double *uy, double *uz)
{
    long n = (long)p->nx * p->ny * p->nz;
    for (long c = 0; c < n; c++) {
        double r = 0.0, jx = 0.0, jy = 0.0, jz = 0.0;
        for (int i = 0; i < Q; i++) {
            double v = f[(long)i * n + c];
            r += v; jx += EX3[i] * v; jy += EY3[i] * v; jz += EZ3[i] * v;
        }
        rho[c] = r; ux[c] = jx; uy[c] = jy; uz[c] = jz;
    }
}

/* Peskin's four-point regularized delta, one axis (cited in Sec. 2.1.2). */
static double peskin(double r)
{
    double a = fabs(r);
    if (a <= 1.0) return (3.0 - 2.0 * a + sqrt(1.0 + 4.0 * a - 4.0 * a * a)) / 8.0;
    if (a <= 2.0) return (5.0 - 2.0 * a - sqrt(-7.0 + 12.0 * a - 4.0 * a * a)) / 8.0;
    return 0.0;
}

double or3_peskin(double r) { return peskin(r); }

/* g(x) = sum_k G_k delta_h(x - X_k) dA with G_k = F n_k, n_k the outward radial
 * normal, dA = 4 pi R^2 / N (Sec. 2.2.2, Eq. (17) on a surface), added to g. */
void or3_spread(const or3_problem *p, const double *X, double *g)
{
    long n = (long)p->nx * p->ny * p->nz;
    double dA = 4.0 * M_PI * p->radius * p->radius / p->n_markers;
    for (int k = 0; k < p->n_markers; k++) {
        double X0 = X[3 * k], Y0 = X[3 * k + 1], Z0 = X[3 * k + 2];
        double nx_ = (X0 - p->cx) / p->radius, ny_ = (Y0 - p->cy) / p->radius, nz_ = (Z0 - p->cz) / p->radius;
        double G[3] = {p->f_normal * nx_, p->f_normal * ny_, p->f_normal * nz_};
        int x0 = (int)floor(X0) - 1, y0 = (int)floor(Y0) - 1, z0 = (int)floor(Z0) - 1;
        for (int dz = 0; dz < 4; dz++)
            for (int dy = 0; dy < 4; dy++)
                for (int dx = 0; dx < 4; dx++) {
                    int x = x0 + dx, y = y0 + dy, z = z0 + dz;
                    double wgt = peskin(x - X0) * peskin(y - Y0) * peskin(z - Z0);
                    long c = ((long)wrap(z, p->nz) * p->ny + wrap(y, p->ny)) * p->nx + wrap(x, p->nx);
                    for (int a = 0; a < 3; a++) g[a * n + c] += G[a] * wgt * dA;
                }
    }
}

static double phi(const or3_problem *p, double x, double y, double z)
{
    return (x - p->cx) * (x - p->cx) + (y - p->cy) * (y - p->cy) + (z - p->cz) * (z - p->cz) -
           p->radius * p->radius;
}

/* Cut links of the sphere's level set phi = |x - c|^2 - R^2 (phi < 0 inside):
 * counts every (x, i) with phi(x) and phi(x + e_i) on different sides. */
long or3_count_cut_links(const or3_problem *p)
{
    long n = 0;
    for (int z = 0; z < p->nz; z++)
        for (int y = 0; y < p->ny; y++)
            for (int x = 0; x < p->nx; x++)
                for (int i = 1; i < Q; i++) {
                    int inP = phi(p, x, y, z) < 0.0;
                    int inQ = phi(p, x + EX3[i], y + EY3[i], z + EZ3[i]) < 0.0;
                    n += inP != inQ;
                }
    return n;
}

/* One step:
 *   1. moments of f^n and the force: body force plus (IB-LBM) the spread F n;
 *   2. SRT collision f* = f - (f - f_eq)/tau + w_i e_i.g / c_s^2;
 *   3. stream f_i(x) = f*_i(x - e_i) + sigma w_i [[p]] / c_s^2 on every link
 *      x - e_i -> x that the level set cuts (II-LBM; sigma = +1 from the
 *      interior), periodic in all three axes. */
int or3_step(const or3_problem *p, double *f, const double *X)
{
    int nx = p->nx, ny = p->ny, nz = p->nz;
    long n = (long)nx * ny * nz;
    double *g = calloc(3 * n, sizeof(double)), *fp = malloc((size_t)Q * n * sizeof(double));
    for (long c = 0; c < n; c++) { g[c] = p->body[0]; g[n + c] = p->body[1]; g[2 * n + c] = p->body[2]; }
    if (p->force_mode == 1 && p->n_markers > 0) or3_spread(p, X, g);
    for (long c = 0; c < n; c++) {
        double fn[Q], r = 0.0, jx = 0.0, jy = 0.0, jz = 0.0, feq[Q];
        for (int i = 0; i < Q; i++) {
            fn[i] = f[(long)i * n + c];
            r += fn[i]; jx += EX3[i] * fn[i]; jy += EY3[i] * fn[i]; jz += EZ3[i] * fn[i];
        }
        or3_equilibrium(r, jx, jy, jz, feq);
        double fs[Q];
        if (p->collision == 1) {
            /* m = M f, m_eq = M f_eq, m* = m - S (m - m_eq), f* = M^-1 m*, with
             * M^-1 = M^T diag(1 / |row k|^2) for the orthogonal rows */
            double dm[Q];
            for (int k = 0; k < Q; k++) {
                double a = 0.0, nk = 0.0;
                for (int i = 0; i < Q; i++) {
                    const double b = basis3(k, EX3[i], EY3[i], EZ3[i]);
                    a += b * (fn[i] - feq[i]);
                    nk += b * b;
                }
                dm[k] = p->s[k] * a / nk;
            }
            for (int i = 0; i < Q; i++) {
                double a = 0.0;
                for (int k = 0; k < Q; k++) a += basis3(k, EX3[i], EY3[i], EZ3[i]) * dm[k];
                fs[i] = fn[i] - a;
            }
        } else {
            for (int i = 0; i < Q; i++) fs[i] = fn[i] - (fn[i] - feq[i]) / p->tau;
        }
        for (int i = 0; i < Q; i++)
            fp[(long)i * n + c] = fs[i] +
                                  wt3(i) * (EX3[i] * g[c] + EY3[i] * g[n + c] + EZ3[i] * g[2 * n + c]) / CS2;
    }
    for (int i = 0; i < Q; i++)
        for (int z = 0; z < nz; z++)
            for (int y = 0; y < ny; y++)
                for (int x = 0; x < nx; x++) {
                    int xs = x - EX3[i], ys = y - EY3[i], zs = z - EZ3[i];
                    double v = fp[id3(p, i, wrap(xs, nx), wrap(ys, ny), wrap(zs, nz))];
                    if (p->force_mode == 0) {
                        int inP = phi(p, xs, ys, zs) < 0.0, inQ = phi(p, x, y, z) < 0.0;
                        if (inP != inQ) v += (inP ? 1.0 : -1.0) * wt3(i) * p->f_normal / CS2;
                    }
                    f[id3(p, i, x, y, z)] = v;
                }
    free(g); free(fp);
    return 0;
}

int or3_run(const or3_problem *p, double *f, const double *X, int steps)
{
    for (int s = 0; s < steps; s++) or3_step(p, f, X);
    return 0;
}

int or3_sizeof_problem(void) { return (int)sizeof(or3_problem); }

/* ------------------------------------------------------------------------
 * A fixed closed triangulated surface (reading R29): the jump conditions of
 * Sec. 3.1 (Eq. (32)) and Sec. 3.2 (Eq. (47)) on the links that cross a
 * triangle mesh, the surface form the paper's conclusion asks of a
 * three-dimensional extension.
 *
 * Vertices are snapped to multiples of 2^-16; every side test is an exact
 * integer determinant.  Ties (a node on a face's plane, a link through an
 * edge or a vertex) are broken by translating the lattice by (e, e^2, e^3)
 * with e -> 0+, which keeps a closed surface closed: every perturbed link
 * meets it in exactly one triangle per crossing.  A link that ends on an
 * edge may clip it (in through one face, out through the other): two
 * records of opposite sigma at the same point, whose jumps cancel.  Triangles are (a, b, c)
 * counter-clockwise seen from outside, so (b - a) x (c - a) points out.
 * A link is P -> P + e_i, keyed by its sending node P; sigma = +1 when P is
 * inside.  [[p]] at the crossing is the barycentric interpolation of the
 * vertex values, the weight of a vertex proportional to the signed volume
 * the link spans with the opposite edge.
 * ---------------------------------------------------------------------- */
typedef __int128 i128;

static int64_t snap16(double v) { return (int64_t)llrint(v * 65536.0); }

static int sgn128(i128 v) { return (v > 0) - (v < 0); }

/* det[u, v, w] = u . (v x w) */
static i128 det3(const int64_t *u, const int64_t *v, const int64_t *w)
{
    return (i128)u[0] * ((i128)v[1] * w[2] - (i128)v[2] * w[1]) -
           (i128)u[1] * ((i128)v[0] * w[2] - (i128)v[2] * w[0]) +
           (i128)u[2] * ((i128)v[0] * w[1] - (i128)v[1] * w[0]);
}

static void sub3(const int64_t *a, const int64_t *b, int64_t *out)
{
    for (int k = 0; k < 3; k++) out[k] = a[k] - b[k];
}

/* Side of the perturbed point P + t of the plane through A, B, C: the sign of
 * det[B - A, C - A, P - A] + t . ((B - A) x (C - A)). */
static int plane_side(const int64_t *A, const int64_t *B, const int64_t *C, const int64_t *P)
{
    int64_t u[3], v[3], w[3];
    sub3(B, A, u); sub3(C, A, v); sub3(P, A, w);
    int s = sgn128(det3(u, v, w));
    if (s) return s;
    i128 n[3] = {(i128)u[1] * v[2] - (i128)u[2] * v[1], (i128)u[2] * v[0] - (i128)u[0] * v[2],
                 (i128)u[0] * v[1] - (i128)u[1] * v[0]};
    for (int k = 0; k < 3; k++)
        if (n[k]) return sgn128(n[k]);
    return 0;
}

/* Orientation of the edge A -> B seen along the perturbed link P -> R:
 * det[R - P, A - P, B - P] + t . ((R - P) x (B - A)); *raw gets the
 * unperturbed determinant (the barycentric weight). */
static int edge_side(const int64_t *P, const int64_t *R, const int64_t *A, const int64_t *B, i128 *raw)
{
    int64_t d[3], a[3], b[3], ba[3];
    sub3(R, P, d); sub3(A, P, a); sub3(B, P, b); sub3(B, A, ba);
    *raw = det3(d, a, b);
    int s = sgn128(*raw);
    if (s) return s;
    i128 c[3] = {(i128)d[1] * ba[2] - (i128)d[2] * ba[1], (i128)d[2] * ba[0] - (i128)d[0] * ba[2],
                 (i128)d[0] * ba[1] - (i128)d[1] * ba[0]};
    for (int k = 0; k < 3; k++)
        if (c[k]) return sgn128(c[k]);
    return 0;
}

/* Every cut link of the surface.  rec[k] = {x, y, z, dir, sigma, tri} of the
 * sending node; val[k] = {[[p]], lambda_a, lambda_b, lambda_c}.  Returns the
 * number of links, or -1 when there are more than cap. */
long or3_mesh_links(const or3_problem *p, int nv, const double *X, int nt, const int32_t *tri,
                    const double *pv, int32_t *rec, double *val, long cap)
{
    (void)p;
    int64_t *S = malloc((size_t)3 * nv * sizeof(int64_t));
    for (int k = 0; k < 3 * nv; k++) S[k] = snap16(X[k]);
    long n = 0;
    for (int t = 0; t < nt; t++) {
        const int ia = tri[3 * t], ib = tri[3 * t + 1], ic = tri[3 * t + 2];
        const int64_t *A = S + 3 * ia, *B = S + 3 * ib, *C = S + 3 * ic;
        int lo[3], hi[3];
        for (int k = 0; k < 3; k++) {
            int64_t mn = A[k], mx = A[k];
            if (B[k] < mn) mn = B[k];
            if (C[k] < mn) mn = C[k];
            if (B[k] > mx) mx = B[k];
            if (C[k] > mx) mx = C[k];
            lo[k] = (int)floor((double)mn / 65536.0) - 1;
            hi[k] = (int)ceil((double)mx / 65536.0) + 1;
        }
        for (int z = lo[2]; z <= hi[2]; z++)
            for (int y = lo[1]; y <= hi[1]; y++)
                for (int x = lo[0]; x <= hi[0]; x++)
                    for (int i = 1; i < Q; i++) {
                        const int64_t P[3] = {(int64_t)x << 16, (int64_t)y << 16, (int64_t)z << 16};
                        const int64_t Qn[3] = {(int64_t)(x + EX3[i]) << 16, (int64_t)(y + EY3[i]) << 16,
                                               (int64_t)(z + EZ3[i]) << 16};
                        const int sp = plane_side(A, B, C, P), sq = plane_side(A, B, C, Qn);
                        if (sp == sq) continue;
                        i128 wc, wa, wb;
                        const int e1 = edge_side(P, Qn, A, B, &wc);
                        const int e2 = edge_side(P, Qn, B, C, &wa);
                        const int e3 = edge_side(P, Qn, C, A, &wb);
                        if (!(e1 == e2 && e2 == e3)) continue;
                        if (n >= cap) { free(S); return -1; }
                        const double la = (double)wa, lb = (double)wb, lc = (double)wc;
                        const double s = la + lb + lc;
                        int32_t *r = rec + 6 * n;
                        r[0] = x; r[1] = y; r[2] = z; r[3] = i; r[4] = sp < 0 ? 1 : -1; r[5] = t;
                        double *v = val + 4 * n;
                        v[1] = la / s; v[2] = lb / s; v[3] = lc / s;
                        v[0] = (la * pv[ia] + lb * pv[ib] + lc * pv[ic]) / s;
                        n++;
                    }
    }
    free(S);
    return n;
}

/* Steps with the surface's jumps: each is the step above (no sphere), then
 * f_i(P + e_i) += sigma w_i [[p]] / c_s^2 on every cut link.  The surface is
 * fixed, so its links are found once. */
int or3_run_mesh(const or3_problem *p, double *f, int nv, const double *X, int nt, const int32_t *tri,
                 const double *pv, int steps)
{
    long cap = 64L * nt + 4096;
    int32_t *rec = malloc((size_t)6 * cap * sizeof(int32_t));
    double *val = malloc((size_t)4 * cap * sizeof(double));
    long n = or3_mesh_links(p, nv, X, nt, tri, pv, rec, val, cap);
    if (n < 0) { free(rec); free(val); return -1; }
    for (int s = 0; s < steps; s++) {
        or3_step(p, f, NULL);
        for (long k = 0; k < n; k++) {
            const int32_t *r = rec + 6 * k;
            const int i = r[3];
            const int x = wrap(r[0] + EX3[i], p->nx), y = wrap(r[1] + EY3[i], p->ny),
                      z = wrap(r[2] + EZ3[i], p->nz);
            f[id3(p, i, x, y, z)] += r[4] * wt3(i) * val[4 * k] / CS2;
        }
    }
    free(rec); free(val);
    return 0;
}

int or3_step_mesh(const or3_problem *p, double *f, int nv, const double *X, int nt, const int32_t *tri,
                  const double *pv)
{
    return or3_run_mesh(p, f, nv, X, nt, tri, pv, 1);
}

/* ------------------------------------------------------------------------
 * A deformable closed triangulated membrane under surface tension gamma
 * (reading R31): the three-dimensional counterpart of the flexible interface
 * of Sec. 2.1 and Sec. 3.2, stepped in the paper's order:
 *   1. U_v = sum_x u^n(x) delta_h(x - X_v), u from the moments of f^n;
 *   2. the force on the fluid at vertex v, G_v = -gamma dA/dX_v (A the total
 *      area), the vertex area A_v (a third of the adjacent triangles), the
 *      outward normal n_v (area-weighted), [[p]]_v = G_v . n_v / A_v and the
 *      tangential part G_v - (G_v . n_v) n_v;
 *   3. the tangential parts spread as g(x) = sum_v Gt_v delta_h(x - X_v);
 *   4. the cut links of the surface at X^n carry [[p]] (as above);
 *   5. collision with g, streaming, the jumps;
 *   6. X^{n+1} = X^n + U^n.
 * ---------------------------------------------------------------------- */

/* dA/da of a triangle (a, b, c) is (1/2) nhat x (c - b), and cyclically. */
int or3_membrane_forces(int nv, const double *X, int nt, const int32_t *tri, double gamma, double *G,
                        double *nrm, double *Av, double *jp, double *Gt)
{
    memset(G, 0, sizeof(double) * 3 * nv);
    memset(nrm, 0, sizeof(double) * 3 * nv);
    memset(Av, 0, sizeof(double) * nv);
    for (int t = 0; t < nt; t++) {
        const int v[3] = {tri[3 * t], tri[3 * t + 1], tri[3 * t + 2]};
        const double *a = X + 3 * v[0], *b = X + 3 * v[1], *c = X + 3 * v[2];
        double u[3], w[3], N[3];
        for (int k = 0; k < 3; k++) { u[k] = b[k] - a[k]; w[k] = c[k] - a[k]; }
        N[0] = u[1] * w[2] - u[2] * w[1];
        N[1] = u[2] * w[0] - u[0] * w[2];
        N[2] = u[0] * w[1] - u[1] * w[0];
        const double len = sqrt(N[0] * N[0] + N[1] * N[1] + N[2] * N[2]);
        if (!(len > 0.0)) return -1;
        const double nh[3] = {N[0] / len, N[1] / len, N[2] / len};
        for (int j = 0; j < 3; j++) {
            const double *p = X + 3 * v[(j + 1) % 3], *q = X + 3 * v[(j + 2) % 3];
            const double e[3] = {q[0] - p[0], q[1] - p[1], q[2] - p[2]};
            const double dA[3] = {0.5 * (nh[1] * e[2] - nh[2] * e[1]), 0.5 * (nh[2] * e[0] - nh[0] * e[2]),
                                  0.5 * (nh[0] * e[1] - nh[1] * e[0])};
            for (int k = 0; k < 3; k++) {
                G[3 * v[j] + k] -= gamma * dA[k];
                nrm[3 * v[j] + k] += N[k];
            }
            Av[v[j]] += len / 6.0;
        }
    }
    for (int i = 0; i < nv; i++) {
        double *n = nrm + 3 * i;
        const double l = sqrt(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]);
        for (int k = 0; k < 3; k++) n[k] /= l;
        const double *g = G + 3 * i;
        const double gn = g[0] * n[0] + g[1] * n[1] + g[2] * n[2];
        jp[i] = gn / Av[i];
        for (int k = 0; k < 3; k++) Gt[3 * i + k] = g[k] - gn * n[k];
    }
    return 0;
}

/* U_v = sum over the 4 x 4 x 4 nodes around X_v of u(x) delta_h(x - X_v),
 * u = sum e_i f_i of the state f (which holds f^n, jumps included). */
void or3_interp(const or3_problem *p, const double *f, int nv, const double *X, double *U)
{
    long n = (long)p->nx * p->ny * p->nz;
    for (int v = 0; v < nv; v++) {
        const double X0 = X[3 * v], Y0 = X[3 * v + 1], Z0 = X[3 * v + 2];
        const int x0 = (int)floor(X0) - 1, y0 = (int)floor(Y0) - 1, z0 = (int)floor(Z0) - 1;
        double acc[3] = {0.0, 0.0, 0.0};
        for (int dz = 0; dz < 4; dz++)
            for (int dy = 0; dy < 4; dy++)
                for (int dx = 0; dx < 4; dx++) {
                    const int x = wrap(x0 + dx, p->nx), y = wrap(y0 + dy, p->ny), z = wrap(z0 + dz, p->nz);
                    const double wgt = peskin(x0 + dx - X0) * peskin(y0 + dy - Y0) * peskin(z0 + dz - Z0);
                    const long c = ((long)z * p->ny + y) * p->nx + x;
                    double jx = 0.0, jy = 0.0, jz = 0.0;
                    for (int i = 0; i < Q; i++) {
                        const double fv = f[(long)i * n + c];
                        jx += EX3[i] * fv; jy += EY3[i] * fv; jz += EZ3[i] * fv;
                    }
                    acc[0] += jx * wgt; acc[1] += jy * wgt; acc[2] += jz * wgt;
                }
        for (int k = 0; k < 3; k++) U[3 * v + k] = acc[k];
    }
}

/* One step of the body force, the force field g (added to the body force),
 * the collision and the streaming: the step above with g given. */
static void step_with_field(const or3_problem *p, double *f, const double *gext)
{
    int nx = p->nx, ny = p->ny, nz = p->nz;
    long n = (long)nx * ny * nz;
    double *fp = malloc((size_t)Q * n * sizeof(double));
    double M[Q][Q], nk[Q];
    for (int k = 0; k < Q; k++) {
        nk[k] = 0.0;
        for (int i = 0; i < Q; i++) { M[k][i] = basis3(k, EX3[i], EY3[i], EZ3[i]); nk[k] += M[k][i] * M[k][i]; }
    }
    for (long c = 0; c < n; c++) {
        double fn[Q], r = 0.0, jx = 0.0, jy = 0.0, jz = 0.0, feq[Q], fs[Q];
        for (int i = 0; i < Q; i++) {
            fn[i] = f[(long)i * n + c];
            r += fn[i]; jx += EX3[i] * fn[i]; jy += EY3[i] * fn[i]; jz += EZ3[i] * fn[i];
        }
        or3_equilibrium(r, jx, jy, jz, feq);
        if (p->collision == 1) {
            double dm[Q];
            for (int k = 0; k < Q; k++) {
                double a = 0.0;
                for (int i = 0; i < Q; i++) a += M[k][i] * (fn[i] - feq[i]);
                dm[k] = p->s[k] * a / nk[k];
            }
            for (int i = 0; i < Q; i++) {
                double a = 0.0;
                for (int k = 0; k < Q; k++) a += M[k][i] * dm[k];
                fs[i] = fn[i] - a;
            }
        } else {
            for (int i = 0; i < Q; i++) fs[i] = fn[i] - (fn[i] - feq[i]) / p->tau;
        }
        const double gx = p->body[0] + gext[c], gy = p->body[1] + gext[n + c], gz = p->body[2] + gext[2 * n + c];
        for (int i = 0; i < Q; i++)
            fp[(long)i * n + c] = fs[i] + wt3(i) * (EX3[i] * gx + EY3[i] * gy + EZ3[i] * gz) / CS2;
    }
    for (int i = 0; i < Q; i++)
        for (int z = 0; z < nz; z++)
            for (int y = 0; y < ny; y++)
                for (int x = 0; x < nx; x++)
                    f[id3(p, i, x, y, z)] = fp[id3(p, i, wrap(x - EX3[i], nx), wrap(y - EY3[i], ny), wrap(z - EZ3[i], nz))];
    free(fp);
}

/* Steps of a triangulated surface, law 0: the membrane under tension gamma,
 * X (3 nv) advanced in place; law 2: the same membrane under IB-LBM (the whole
 * G_v spread, no jumps; Sec. 2.2.2); law 1: a fixed rigid surface with the direct
 * forcing of Sec. 2.1.2 (Eq. (9) with eta = 1 and U^D = 0, reading R32), the
 * force on the fluid at a vertex G_v = (U^D - U_v) A_v, X unchanged.  U (3 nv)
 * and F (3) (either may be NULL) receive the last step's vertex velocities and
 * the force on the surface, F = -sum_v G_v (Sec. 2.1.3).  Returns -1 when the
 * surface degenerates or overflows the link buffer. */
static int run_surface_ud(const or3_problem *p, double *f, int nv, double *X, int nt, const int32_t *tri, int law,
                          double gamma, int steps, double *Uout, double *Fout, const double *UD, double *Gout);

int or3_run_surface(const or3_problem *p, double *f, int nv, double *X, int nt, const int32_t *tri, int law,
                    double gamma, int steps, double *Uout, double *Fout)
{
    return run_surface_ud(p, f, nv, X, nt, tri, law, gamma, steps, Uout, Fout, NULL, NULL);
}

/* As above; the rigid law holds the vertices at UD (3 nv, NULL: rest), and
 * Gout (3 nv, may be NULL) receives the last step's G. */
static int run_surface_ud(const or3_problem *p, double *f, int nv, double *X, int nt, const int32_t *tri, int law,
                          double gamma, int steps, double *Uout, double *Fout, const double *UD, double *Gout)
{
    long n = (long)p->nx * p->ny * p->nz;
    long cap = 64L * nt + 4096;
    double *G = malloc(sizeof(double) * 3 * nv), *nrm = malloc(sizeof(double) * 3 * nv);
    double *Av = malloc(sizeof(double) * nv), *jp = malloc(sizeof(double) * nv);
    double *Gt = malloc(sizeof(double) * 3 * nv), *U = malloc(sizeof(double) * 3 * nv);
    double *g = malloc(sizeof(double) * 3 * n);
    int32_t *rec = malloc((size_t)6 * cap * sizeof(int32_t));
    double *val = malloc((size_t)4 * cap * sizeof(double));
    int rc = 0;
    for (int s = 0; s < steps && rc == 0; s++) {
        or3_interp(p, f, nv, X, U);
        if (or3_membrane_forces(nv, X, nt, tri, law == 1 ? 0.0 : gamma, G, nrm, Av, jp, Gt)) { rc = -1; break; }
        if (law == 1)
            for (int v = 0; v < nv; v++) {
                const double *n = nrm + 3 * v;
                double g3[3];
                for (int k = 0; k < 3; k++) g3[k] = ((UD ? UD[3 * v + k] : 0.0) - U[3 * v + k]) * Av[v];
                const double gn = g3[0] * n[0] + g3[1] * n[1] + g3[2] * n[2];
                jp[v] = gn / Av[v];
                for (int k = 0; k < 3; k++) {
                    G[3 * v + k] = g3[k];
                    Gt[3 * v + k] = g3[k] - gn * n[k];
                }
            }
        if (law == 2)
            for (int v = 0; v < nv; v++) {
                jp[v] = 0.0;
                for (int k = 0; k < 3; k++) Gt[3 * v + k] = G[3 * v + k];
            }
        if (Fout) {
            Fout[0] = Fout[1] = Fout[2] = 0.0;
            for (int v = 0; v < nv; v++)
                for (int k = 0; k < 3; k++) Fout[k] -= G[3 * v + k];
        }
        memset(g, 0, sizeof(double) * 3 * n);
        for (int v = 0; v < nv; v++) {
            const double X0 = X[3 * v], Y0 = X[3 * v + 1], Z0 = X[3 * v + 2];
            const int x0 = (int)floor(X0) - 1, y0 = (int)floor(Y0) - 1, z0 = (int)floor(Z0) - 1;
            for (int dz = 0; dz < 4; dz++)
                for (int dy = 0; dy < 4; dy++)
                    for (int dx = 0; dx < 4; dx++) {
                        const double wgt = peskin(x0 + dx - X0) * peskin(y0 + dy - Y0) * peskin(z0 + dz - Z0);
                        const long c = ((long)wrap(z0 + dz, p->nz) * p->ny + wrap(y0 + dy, p->ny)) * p->nx +
                                       wrap(x0 + dx, p->nx);
                        for (int k = 0; k < 3; k++) g[k * n + c] += Gt[3 * v + k] * wgt;
                    }
        }
        /* IB-LBM membrane (reading R18, as in two dimensions): the vertices
         * move with the velocity of the distributions after the step's force,
         * u + g, so the spread force and the body force join U_v */
        if (law == 2)
            for (int v = 0; v < nv; v++) {
                const double X0 = X[3 * v], Y0 = X[3 * v + 1], Z0 = X[3 * v + 2];
                const int x0 = (int)floor(X0) - 1, y0 = (int)floor(Y0) - 1, z0 = (int)floor(Z0) - 1;
                double acc[3] = {p->body[0], p->body[1], p->body[2]};
                for (int dz = 0; dz < 4; dz++)
                    for (int dy = 0; dy < 4; dy++)
                        for (int dx = 0; dx < 4; dx++) {
                            const double wgt = peskin(x0 + dx - X0) * peskin(y0 + dy - Y0) * peskin(z0 + dz - Z0);
                            const long c = ((long)wrap(z0 + dz, p->nz) * p->ny + wrap(y0 + dy, p->ny)) * p->nx +
                                           wrap(x0 + dx, p->nx);
                            for (int k = 0; k < 3; k++) acc[k] += g[k * n + c] * wgt;
                        }
                for (int k = 0; k < 3; k++) U[3 * v + k] += acc[k];
            }
        const long nl = law == 2 ? 0 : or3_mesh_links(p, nv, X, nt, tri, jp, rec, val, cap);
        if (nl < 0) { rc = -1; break; }
        step_with_field(p, f, g);
        for (long k = 0; k < nl; k++) {
            const int32_t *r = rec + 6 * k;
            const int i = r[3];
            const int x = wrap(r[0] + EX3[i], p->nx), y = wrap(r[1] + EY3[i], p->ny), z = wrap(r[2] + EZ3[i], p->nz);
            f[id3(p, i, x, y, z)] += r[4] * wt3(i) * val[4 * k] / CS2;
        }
        if (law != 1)
            for (int k = 0; k < 3 * nv; k++) X[k] += U[k];
    }
    if (Uout && rc == 0) memcpy(Uout, U, sizeof(double) * 3 * nv);
    if (Gout && rc == 0) memcpy(Gout, G, sizeof(double) * 3 * nv);
    free(G); free(nrm); free(Av); free(jp); free(Gt); free(U); free(g); free(rec); free(val);
    return rc;
}

int or3_run_membrane(const or3_problem *p, double *f, int nv, double *X, int nt, const int32_t *tri,
                     double gamma, int steps, double *Uout)
{
    return or3_run_surface(p, f, nv, X, nt, tri, 0, gamma, steps, Uout, NULL);
}

/* ------------------------------------------------------------------------
 * A free rigid sphere (reading R33): the rigid-body update of Sec. 2.3 in
 * three dimensions.  The vertices keep their offsets r_v from the centre (a
 * rotation leaves a sphere's surface the same set) and move with it.  Per
 * step:
 *   1. the surface step with U^D_v = U + W x r_v;
 *   2. F = -sum G_v + rho_f V_s (U^n - U^{n-1}),
 *      T = -sum r_v x G_v + (I_s / rho*) (W^n - W^{n-1}),
 *      with rho_f = 1, V_s = 4 pi R^3 / 3, m = rho* V_s, I_s = 2 m R^2 / 5;
 *   3. a^{n+1} = F / m, U^{n+1} = U^n + a^{n+1},
 *      c^{n+1} = c^n + U^n + (a^n + a^{n+1}) / 2; w^{n+1} = T / I_s,
 *      W^{n+1} = W^n + w^{n+1}.
 * body[21] = {c[3], U[3], a[3], W[3], wdot[3], Uprev[3], Wprev[3]}, updated in
 * place; F and T (3 each, may be NULL) receive the last step's force and
 * torque.  The first step takes Uprev = U, Wprev = W.
 * ---------------------------------------------------------------------- */
int or3_run_free_sphere(const or3_problem *p, double *f, int nv, double *X, int nt, const int32_t *tri,
                        double radius, double rho_star, double *body, int steps, double *Fout, double *Tout)
{
    double *c = body, *Ub = body + 3, *a = body + 6, *W = body + 9, *wd = body + 12, *Up = body + 15,
           *Wp = body + 18;
    const double Vs = 4.0 * M_PI * radius * radius * radius / 3.0, m = rho_star * Vs,
                 Is = 0.4 * m * radius * radius;
    double *r = malloc(sizeof(double) * 3 * nv), *UD = malloc(sizeof(double) * 3 * nv),
           *G = malloc(sizeof(double) * 3 * nv);
    for (int v = 0; v < nv; v++)
        for (int k = 0; k < 3; k++) r[3 * v + k] = X[3 * v + k] - c[k];
    int rc = 0;
    for (int s = 0; s < steps && rc == 0; s++) {
        for (int v = 0; v < nv; v++) {
            const double *q = r + 3 * v;
            UD[3 * v] = Ub[0] + W[1] * q[2] - W[2] * q[1];
            UD[3 * v + 1] = Ub[1] + W[2] * q[0] - W[0] * q[2];
            UD[3 * v + 2] = Ub[2] + W[0] * q[1] - W[1] * q[0];
        }
        rc = run_surface_ud(p, f, nv, X, nt, tri, 1, 0.0, 1, NULL, NULL, UD, G);
        if (rc) break;
        double F[3] = {0.0, 0.0, 0.0}, T[3] = {0.0, 0.0, 0.0};
        for (int v = 0; v < nv; v++) {
            const double *q = r + 3 * v, *g = G + 3 * v;
            for (int k = 0; k < 3; k++) F[k] -= g[k];
            T[0] -= q[1] * g[2] - q[2] * g[1];
            T[1] -= q[2] * g[0] - q[0] * g[2];
            T[2] -= q[0] * g[1] - q[1] * g[0];
        }
        for (int k = 0; k < 3; k++) {
            F[k] += Vs * (Ub[k] - Up[k]);
            T[k] += Is / rho_star * (W[k] - Wp[k]);
        }
        for (int k = 0; k < 3; k++) {
            const double an = F[k] / m, wn = T[k] / Is;
            Up[k] = Ub[k];
            Wp[k] = W[k];
            const double dc = Ub[k] + 0.5 * (a[k] + an);
            c[k] += dc;
            for (int v = 0; v < nv; v++) X[3 * v + k] += dc;
            Ub[k] += an;
            a[k] = an;
            W[k] += wn;
            wd[k] = wn;
        }
        if (Fout) memcpy(Fout, F, sizeof F);
        if (Tout) memcpy(Tout, T, sizeof T);
    }
    free(r); free(UD); free(G);
    return rc;
}
