/*
 * Plain FP64 CPU oracle of the D2Q9 immersed interface-lattice Boltzmann
 * method (II-LBM) of Qin, Kolahdouz & Griffith, "An immersed interface-lattice
 * Boltzmann method for fluid-structure interaction" (arXiv:2003.12186).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may call, link or
 * load this file; it exists so that tests, the smoke check and the CPU leg of
 * the benchmark can compare the GPU library against a slow, plain, obviously
 * correct implementation written from the paper.  It shares no code, header,
 * table or helper with the GPU library.
 *
 * Everything is double precision, one plain loop per equation, in the order
 * of the paper's algorithm.  Lattice units throughout (dx = dt = 1, Sec. 2.2).
 * Field layout: f[i][y][x] with x fastest; markers X[k][2] interleaved.
 *
 * Readings taken where the paper is silent (each is listed with its reason in
 * the design notes of the repository):
 *  R1  moments sum over all nine populations including f_0 (the derivation in
 *      Sec. 3.1 sums over every i);
 *  R2  D2Q9 numbering e0=(0,0), e1=(1,0), e2=(0,1), e3=(-1,0), e4=(0,-1),
 *      e5=(1,1), e6=(-1,1), e7=(-1,-1), e8=(1,-1); consistent with the P1/P2
 *      example at the end of Sec. 3.2;
 *  R3  MRT moment basis of Lallemand & Luo (cited in Sec. 2.1.1), m_eq = M f_eq
 *      with the He-Luo equilibrium, so MRT with every rate 1/tau equals SRT;
 *  R4  collide at the node, then stream (force and RHS at the upstream node);
 *  R5  jumps and tangential force of step n use the interface at X^n;
 *  R6  a link from the interior to the exterior adds +[[f_i]], the reverse
 *      link adds -[[f_i]], several crossings add up;
 *  R7  markers counter-clockwise, outward normal n = rot(-90 deg) of the
 *      central chord X_{k+1}-X_{k-1};
 *  R8  |dX/ds| at a membrane marker = mean length of its two chords / Delta X;
 *  R9  the tangential part is G - (G.n) n;
 *  R10 the flexible interface is the closed polygon through the markers, snapped
 *      to a 2^-16 grid, tested with exact integer orientations and the node
 *      perturbation tie rule; [[p]] is linear along each chord;
 *  R11 marker velocity from u = sum e_i f_i of the pre-collision field
 *      (II-LBM);
 *  R18 the IB-LBM comparison modes (the whole force spread, no jumps) move a
 *      membrane with the scheme's own velocity taken from the distributions
 *      after the step's collision and force term (momentum sum e_i f_i + g):
 *      u = sum e_i f_i + g under the simple term, (sum e_i f_i + 3 g / 2) / rho
 *      under Guo's; Table 2 fixes this: it is the reading under which both
 *      IB-LBM columns lose area at the printed rates;
 *  R12 non-equilibrium extrapolation on non-periodic sides, corners as walls
 *      (a uniform inflow side takes u_b = (u_max, 0));
 *  R27 (geometry 1) the membrane is the periodic cubic spline through the
 *      markers in the marker index; crossings are the roots of a cubic found
 *      by a fixed bisection after a control-point hull test, [[p]] at a crossing from the spline normal and
 *      |dX/ds| with G linear between the markers;
 *  R24 under Guo's force term (the comparison method of Sec. 2.2.2) the
 *      collision uses the compressible equilibrium and the velocity
 *      u = (sum e_i f_i + g/2) / rho the paper gives with it, g the whole
 *      Eulerian force (g_par plus the body force for II-LBM, Sec. 3.2); the
 *      II-LBM markers move with that u (R11 holds for the simple force term,
 *      R18 for the IB-LBM modes); the direct-forcing u* carries the body force
 *      only.
 */
#define _GNU_SOURCE
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------ */
/* Problem description (the oracle's own struct; filled from Python).        */
/* ------------------------------------------------------------------------ */
enum { OR_SRT = 0, OR_MRT = 1 };
enum { OR_PERIODIC = 0, OR_WALL = 1, OR_INLET = 2, OR_OUTLET = 3, OR_INLET_UNIFORM = 4 };
/* Interfaces: a spring membrane, a fixed circle with direct forcing, and a
 * fixed circle with a prescribed uniform normal force (Sec. 4.1). */
enum { OR_IF_NONE = 0, OR_IF_MEMBRANE = 1, OR_IF_RIGID = 2, OR_IF_NORMAL = 3 };
/* Force modes: II-LBM (jumps, tangential force in the simple term, the
 * paper's method); IB-LBM (the full force spread, no jumps) with the simple
 * term or Guo's term; II-LBM with Guo's term of the tangential force
 * (Sec. 3.2, the remark on Guo's terms). */
enum { OR_II_LBM = 0, OR_IB_LBM = 1, OR_IB_LBM_GUO = 2, OR_II_LBM_GUO = 3 };

typedef struct {
    int32_t nx, ny;
    double tau;
    int32_t collision;
    double s[9];          /* MRT rates in moment order (rho,e,eps,jx,qx,jy,qy,pxx,pxy) */
    int32_t bc[4];        /* x-low, x-high, y-low, y-high */
    double u_max;         /* inlet parabola peak */
    double u_wall[4];     /* tangential wall speed per side */
    double body[2];       /* uniform Eulerian body force */
    int32_t interface;
    int32_t force_mode;
    int32_t n_markers;
    double kappa, dX;
    double cx, cy, radius; /* rigid circle */
    double f_normal;       /* prescribed force per unit length along the outward normal */
    /* a moving rigid circle (Sec. 2.3): the body velocity U_c, W that direct
     * forcing drives the markers to (U^D = U_c + W x (X - X_c)), and the
     * orientation theta (marker k sits at angle theta + 2 pi k / N) */
    double ud[3];
    double theta;
    int32_t geometry;      /* membrane representation: 0 polygon (R10), 1 cubic spline (R27) */
    int32_t pad2;
} or_problem;

static int has_jumps(const or_problem *p) { return p->force_mode == OR_II_LBM || p->force_mode == OR_II_LBM_GUO; }
static int uses_guo(const or_problem *p) { return p->force_mode == OR_IB_LBM_GUO || p->force_mode == OR_II_LBM_GUO; }

/* One cut link: source node (x, y), direction i, its sign and where it is cut. */
typedef struct {
    int32_t x, y, dir, sigma, seg, pad;
    double q;      /* fraction along the link from the source node to the cut point */
    double theta;  /* fraction along the interface chord (or marker interval) */
    double jp;     /* [[p]] at the cut point */
} or_link;

/* ------------------------------------------------------------------------ */
/* D2Q9 lattice (Sec. 2.1.1 velocities; Sec. 2.2.1 weights and c_s).        */
/* ------------------------------------------------------------------------ */
static const int EX[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
static const int EY[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
static const double WT[9] = {4.0 / 9.0, 1.0 / 9.0, 1.0 / 9.0, 1.0 / 9.0, 1.0 / 9.0,
                             1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0};
static const double CS2 = 1.0 / 3.0; /* c_s^2, c_s = 1/sqrt(3) */

void or_d2q9(int32_t *ex, int32_t *ey, double *w)
{
    for (int i = 0; i < 9; i++) { ex[i] = EX[i]; ey[i] = EY[i]; w[i] = WT[i]; }
}

static long idx(const or_problem *p, int i, int x, int y)
{
    return ((long)i * p->ny + y) * p->nx + x;
}

/* ------------------------------------------------------------------------ */
/* Equilibrium and moments (Sec. 2.2.1).                                     */
/* ------------------------------------------------------------------------ */

/* He-Luo incompressible equilibrium, Sec. 2.2.1 Eq. (10), written with
 * rho = p / c_s^2:  f_i = w_i [ p/c_s^2 + e.u/c_s^2 + (e.u)^2/(2 c_s^4) - u.u/(2 c_s^2) ]. */
void or_equilibrium(double rho, double ux, double uy, double *feq)
{
    double p = CS2 * rho;
    double uu = ux * ux + uy * uy;
    for (int i = 0; i < 9; i++) {
        double eu = EX[i] * ux + EY[i] * uy;
        feq[i] = WT[i] * (p / CS2 + eu / CS2 + eu * eu / (2.0 * CS2 * CS2) - uu / (2.0 * CS2));
    }
}

/* Pressure and velocity, Sec. 2.2.1 Eqs. (11)-(12), summed over all nine
 * populations (reading R1).  Returns rho = p / c_s^2. */
void or_moments_node(const double *f, double *rho, double *ux, double *uy)
{
    double r = 0.0, jx = 0.0, jy = 0.0;
    for (int i = 0; i < 9; i++) {
        r += f[i];
        jx += EX[i] * f[i];
        jy += EY[i] * f[i];
    }
    *rho = r; *ux = jx; *uy = jy;
}

void or_moments(const or_problem *p, const double *f, double *rho, double *ux, double *uy)
{
#pragma omp parallel for
    for (int y = 0; y < p->ny; y++)
        for (int x = 0; x < p->nx; x++) {
            double fn[9];
            for (int i = 0; i < 9; i++) fn[i] = f[idx(p, i, x, y)];
            long n = (long)y * p->nx + x;
            or_moments_node(fn, &rho[n], &ux[n], &uy[n]);
        }
}

/* ------------------------------------------------------------------------ */
/* Collision (Sec. 2.2.1 SRT and MRT, Sec. 2.2.2 simple force term).         */
/* ------------------------------------------------------------------------ */

/* MRT transform of Lallemand & Luo (reading R3): rows are polynomials of the
 * lattice velocity c = e_i with c2 = |c|^2, in the order
 * (rho, e, eps, jx, qx, jy, qy, pxx, pxy). */
void or_mrt_matrices(double *M, double *Minv)
{
    for (int i = 0; i < 9; i++) {
        double cx = EX[i], cy = EY[i], c2 = cx * cx + cy * cy;
        M[0 * 9 + i] = 1.0;
        M[1 * 9 + i] = -4.0 + 3.0 * c2;
        M[2 * 9 + i] = 4.0 - 10.5 * c2 + 4.5 * c2 * c2;
        M[3 * 9 + i] = cx;
        M[4 * 9 + i] = (-5.0 + 3.0 * c2) * cx;
        M[5 * 9 + i] = cy;
        M[6 * 9 + i] = (-5.0 + 3.0 * c2) * cy;
        M[7 * 9 + i] = cx * cx - cy * cy;
        M[8 * 9 + i] = cx * cy;
    }
    /* The rows are mutually orthogonal, so M^-1 = M^T diag(1 / |row|^2).
     * (A test checks M Minv = I against a general-purpose inverse.) */
    for (int a = 0; a < 9; a++) {
        double nrm = 0.0;
        for (int i = 0; i < 9; i++) nrm += M[a * 9 + i] * M[a * 9 + i];
        for (int i = 0; i < 9; i++) Minv[i * 9 + a] = M[a * 9 + i] / nrm;
    }
}

/* Post-collision populations at one node.
 * SRT: f* = f - (f - f_eq)/tau (Sec. 2.2.1, Eq. (14) with lambda = tau).
 * MRT: f* = f - M^-1 S (M f - M f_eq) (Sec. 2.2.1, Eq. (15)).
 * Then the simple external force term of He et al., + w_i e_i.g / c_s^2
 * (Sec. 2.2.2, Eq. (16)), added in velocity space (also under MRT). */
static void collide_with(const or_problem *p, const double *M, const double *Minv,
                         const double *f, double gx, double gy, double *out)
{
    double rho, ux, uy, feq[9];
    or_moments_node(f, &rho, &ux, &uy);
    or_equilibrium(rho, ux, uy, feq);
    if (p->collision == OR_SRT) {
        for (int i = 0; i < 9; i++) out[i] = f[i] - (f[i] - feq[i]) / p->tau;
    } else {
        double m[9], meq[9], mstar[9];
        for (int a = 0; a < 9; a++) {
            m[a] = 0.0; meq[a] = 0.0;
            for (int i = 0; i < 9; i++) { m[a] += M[a * 9 + i] * f[i]; meq[a] += M[a * 9 + i] * feq[i]; }
            mstar[a] = m[a] - p->s[a] * (m[a] - meq[a]);
        }
        for (int i = 0; i < 9; i++) {
            out[i] = 0.0;
            for (int a = 0; a < 9; a++) out[i] += Minv[i * 9 + a] * mstar[a];
        }
    }
    for (int i = 0; i < 9; i++) out[i] += WT[i] * (EX[i] * gx + EY[i] * gy) / CS2;
}

/* Guo's force distribution without its relaxation factor (Sec. 2.2.2, the
 * bracket of Eq. (SRT_Guo_) and the G~_i of Eq. (MRT_Guo_)):
 *   G~_i = w_i [ (e_i - u)/c_s^2 + (e_i.u) e_i / c_s^4 ] . g */
void or_guo_term(double ux, double uy, double gx, double gy, double *G)
{
    for (int i = 0; i < 9; i++) {
        double eu = EX[i] * ux + EY[i] * uy, eg = EX[i] * gx + EY[i] * gy;
        G[i] = WT[i] * (((EX[i] - ux) * gx + (EY[i] - uy) * gy) / CS2 + eu * eg / (CS2 * CS2));
    }
}

/* Collision with Guo's force term (reading R24): the velocity
 * p/c_s^2 u = sum_i e_i f_i + g/2 and the equilibrium
 * w_i p/c_s^2 [1 + e.u/c_s^2 + (e.u)^2/(2 c_s^4) - u.u/(2 c_s^2)];
 * SRT: f* = f - (f - f_eq)/tau + (1 - 1/(2 tau)) G~;
 * MRT: f* = f - M^-1 S (M f - M f_eq) + M^-1 (I - S/2) M G~. */
static void collide_guo(const or_problem *p, const double *M, const double *Minv,
                        const double *f, double gx, double gy, double *out)
{
    double rho, jx, jy, feq[9], G[9];
    or_moments_node(f, &rho, &jx, &jy);
    double ux = (jx + 0.5 * gx) / rho, uy = (jy + 0.5 * gy) / rho;
    double uu = ux * ux + uy * uy;
    for (int i = 0; i < 9; i++) {
        double eu = EX[i] * ux + EY[i] * uy;
        feq[i] = WT[i] * rho * (1.0 + eu / CS2 + eu * eu / (2.0 * CS2 * CS2) - uu / (2.0 * CS2));
    }
    or_guo_term(ux, uy, gx, gy, G);
    if (p->collision == OR_SRT) {
        for (int i = 0; i < 9; i++)
            out[i] = f[i] - (f[i] - feq[i]) / p->tau + (1.0 - 0.5 / p->tau) * G[i];
        return;
    }
    double m[9], meq[9], mg[9], mstar[9];
    for (int a = 0; a < 9; a++) {
        m[a] = 0.0; meq[a] = 0.0; mg[a] = 0.0;
        for (int i = 0; i < 9; i++) {
            m[a] += M[a * 9 + i] * f[i];
            meq[a] += M[a * 9 + i] * feq[i];
            mg[a] += M[a * 9 + i] * G[i];
        }
        mstar[a] = m[a] - p->s[a] * (m[a] - meq[a]) + (1.0 - 0.5 * p->s[a]) * mg[a];
    }
    for (int i = 0; i < 9; i++) {
        out[i] = 0.0;
        for (int a = 0; a < 9; a++) out[i] += Minv[i * 9 + a] * mstar[a];
    }
}

void or_collide_node(const or_problem *p, const double *f, double gx, double gy, double *out)
{
    double M[81], Minv[81];
    or_mrt_matrices(M, Minv);
    if (uses_guo(p))
        collide_guo(p, M, Minv, f, gx, gy, out);
    else
        collide_with(p, M, Minv, f, gx, gy, out);
}

/* ------------------------------------------------------------------------ */
/* Peskin's four-point regularized delta (cited in Sec. 2.1.2).              */
/* ------------------------------------------------------------------------ */
double or_peskin_phi(double r)
{
    double a = fabs(r);
    if (a <= 1.0) return (3.0 - 2.0 * a + sqrt(1.0 + 4.0 * a - 4.0 * a * a)) / 8.0;
    if (a <= 2.0) return (5.0 - 2.0 * a - sqrt(-7.0 + 12.0 * a - 4.0 * a * a)) / 8.0;
    return 0.0;
}

/* Wrap a lattice index on a periodic axis; on a bounded axis return -1 when out. */
static int wrap_x(const or_problem *p, int x)
{
    if (p->bc[0] == OR_PERIODIC) return ((x % p->nx) + p->nx) % p->nx;
    return (x >= 0 && x < p->nx) ? x : -1;
}
static int wrap_y(const or_problem *p, int y)
{
    if (p->bc[2] == OR_PERIODIC) return ((y % p->ny) + p->ny) % p->ny;
    return (y >= 0 && y < p->ny) ? y : -1;
}

/* Interpolated marker velocity U_k = sum_x u(x) delta_h(x - X_k) dx^2
 * (Sec. 2.2.2, Eq. (20); also U* of Eq. (18)). */
void or_interp(const or_problem *p, const double *ux, const double *uy, const double *X, double *U)
{
    for (int k = 0; k < p->n_markers; k++) {
        double Xk = X[2 * k], Yk = X[2 * k + 1], sx = 0.0, sy = 0.0;
        int x0 = (int)floor(Xk) - 2, y0 = (int)floor(Yk) - 2;
        for (int y = y0; y <= y0 + 5; y++)
            for (int x = x0; x <= x0 + 5; x++) {
                double w = or_peskin_phi(x - Xk) * or_peskin_phi(y - Yk);
                if (w == 0.0) continue;
                int xx = wrap_x(p, x), yy = wrap_y(p, y);
                if (xx < 0 || yy < 0) continue;
                long n = (long)yy * p->nx + xx;
                sx += ux[n] * w;
                sy += uy[n] * w;
            }
        U[2 * k] = sx; U[2 * k + 1] = sy;
    }
}

/* Eulerian force density g(x) += sum_k V_k delta_h(x - X_k) Delta X
 * (Sec. 2.2.2, Eq. (17); the tangential version is Sec. 3.2, Eq. (46)). */
void or_spread(const or_problem *p, const double *X, const double *V, double *gx, double *gy)
{
    for (int k = 0; k < p->n_markers; k++) {
        double Xk = X[2 * k], Yk = X[2 * k + 1];
        int x0 = (int)floor(Xk) - 2, y0 = (int)floor(Yk) - 2;
        for (int y = y0; y <= y0 + 5; y++)
            for (int x = x0; x <= x0 + 5; x++) {
                double w = or_peskin_phi(x - Xk) * or_peskin_phi(y - Yk);
                if (w == 0.0) continue;
                int xx = wrap_x(p, x), yy = wrap_y(p, y);
                if (xx < 0 || yy < 0) continue;
                long n = (long)yy * p->nx + xx;
                gx[n] += V[2 * k] * w * p->dX;
                gy[n] += V[2 * k + 1] * w * p->dX;
            }
    }
}

/* ------------------------------------------------------------------------ */
/* Periodic cubic spline through the markers (reading R27; Sec. 3.2 names a   */
/* cubic spline for flexible interfaces).                                    */
/* ------------------------------------------------------------------------ */

/* Second derivatives M_k of the periodic cubic spline in the marker index:
 * M_{k-1} + 4 M_k + M_{k+1} = 6 (X_{k+1} - 2 X_k + X_{k-1}), one component at a
 * time (stride 2), solved as a cyclic tridiagonal system (Sherman-Morrison
 * around the Thomas algorithm). */
static void spline_second_derivs(int N, const double *X, int comp, double *M)
{
    double *r = malloc(N * sizeof(double)), *y = malloc(N * sizeof(double));
    double *z = malloc(N * sizeof(double)), *cp = malloc(N * sizeof(double));
    double *u = calloc(N, sizeof(double));
    for (int k = 0; k < N; k++) {
        int km = (k + N - 1) % N, kp = (k + 1) % N;
        r[k] = 6.0 * (X[2 * kp + comp] - 2.0 * X[2 * k + comp] + X[2 * km + comp]);
    }
    /* A = T + u v^T with gamma = -4: T_00 = 4 - gamma, T_nn = 4 - 1/gamma,
     * u = (gamma, 0, .., 0, 1), v = (1, 0, .., 0, 1/gamma) */
    double gamma = -4.0;
    u[0] = gamma; u[N - 1] = 1.0;
    for (int pass = 0; pass < 2; pass++) {
        const double *rhs = pass == 0 ? r : u;
        double *out = pass == 0 ? y : z;
        /* Thomas on the tridiagonal T (sub = super = 1) */
        double b0 = 4.0 - gamma;
        cp[0] = 1.0 / b0;
        out[0] = rhs[0] / b0;
        for (int k = 1; k < N; k++) {
            double bk = (k == N - 1) ? 4.0 - 1.0 / gamma : 4.0;
            double den = bk - cp[k - 1];
            cp[k] = 1.0 / den;
            out[k] = (rhs[k] - out[k - 1]) / den;
        }
        for (int k = N - 2; k >= 0; k--) out[k] -= cp[k] * out[k + 1];
    }
    double vy = y[0] + y[N - 1] / gamma, vz = z[0] + z[N - 1] / gamma;
    for (int k = 0; k < N; k++) M[2 * k + comp] = y[k] - vy / (1.0 + vz) * z[k];
    free(r); free(y); free(z); free(cp); free(u);
}

/* Segment k of the spline, S(t) = a + b t + c t^2 + d t^3 on t in [0, 1]:
 * a = X_k, b = X_{k+1} - X_k - (2 M_k + M_{k+1}) / 6, c = M_k / 2,
 * d = (M_{k+1} - M_k) / 6; coef[8] = (ax, ay, bx, by, cx, cy, dx, dy). */
static void spline_segment(int N, const double *X, const double *M, int k, double *coef)
{
    int kp = (k + 1) % N;
    for (int c = 0; c < 2; c++) {
        coef[0 + c] = X[2 * k + c];
        coef[2 + c] = X[2 * kp + c] - X[2 * k + c] - (2.0 * M[2 * k + c] + M[2 * kp + c]) / 6.0;
        coef[4 + c] = 0.5 * M[2 * k + c];
        coef[6 + c] = (M[2 * kp + c] - M[2 * k + c]) / 6.0;
    }
}

void or_spline(const or_problem *p, const double *X, double *M)
{
    spline_second_derivs(p->n_markers, X, 0, M);
    spline_second_derivs(p->n_markers, X, 1, M);
}

static double cubic_at(const double F[4], double t) { return ((F[3] * t + F[2]) * t + F[1]) * t + F[0]; }

/* Crossings of the link P -> P + e with spline segment coef (reading R27).
 * f(t) = e x (S(t) - P) is a cubic; [0, 1] is split at the critical points
 * inside it, each piece with a sign change of f (f >= 0 counts as positive;
 * f(1) is e x (X_{k+1} - P) as the next segment's f(0)) holds one root,
 * found by 64 bisections.  A root at link parameter q in [0, 1) is a
 * crossing; sigma = +1 when f rises through it (P on the interior side).
 * Writes up to 3 (t, q, sigma); returns their count. */
static int spline_link_crossings(const double *coef, const double *Xnext, double px, double py,
                                 int ex, int ey, double *ts, double *qs, int *sg)
{
    /* the segment lies in the hull of its Bezier control points
     * B0 = a, B1 = a + b/3, B2 = a + (2b + c)/3, B3 = X_{k+1}: when e x (B_i - P)
     * has one strict sign for all four, the line of the link misses it */
    double b1x = coef[0] + coef[2] / 3.0, b1y = coef[1] + coef[3] / 3.0;
    double b2x = coef[0] + (2.0 * coef[2] + coef[4]) / 3.0, b2y = coef[1] + (2.0 * coef[3] + coef[5]) / 3.0;
    double bz[4];
    bz[0] = ex * (coef[1] - py) - ey * (coef[0] - px);
    bz[1] = ex * (b1y - py) - ey * (b1x - px);
    bz[2] = ex * (b2y - py) - ey * (b2x - px);
    bz[3] = ex * (Xnext[1] - py) - ey * (Xnext[0] - px);
    if ((bz[0] > 0.0 && bz[1] > 0.0 && bz[2] > 0.0 && bz[3] > 0.0) ||
        (bz[0] < 0.0 && bz[1] < 0.0 && bz[2] < 0.0 && bz[3] < 0.0))
        return 0;
    double F[4];
    F[0] = ex * (coef[1] - py) - ey * (coef[0] - px);
    F[1] = ex * coef[3] - ey * coef[2];
    F[2] = ex * coef[5] - ey * coef[4];
    F[3] = ex * coef[7] - ey * coef[6];
    double f1 = ex * (Xnext[1] - py) - ey * (Xnext[0] - px);
    /* critical points: 3 F3 t^2 + 2 F2 t + F1 = 0 */
    double br[4];
    int nb = 0;
    br[nb++] = 0.0;
    double A = 3.0 * F[3], Bq = 2.0 * F[2], Cq = F[1];
    double r1 = -1.0, r2 = -1.0;
    if (A == 0.0) {
        if (Bq != 0.0) r1 = -Cq / Bq;
    } else {
        double disc = Bq * Bq - 4.0 * A * Cq;
        if (disc > 0.0) {
            double sq = sqrt(disc);
            double qq = Bq >= 0.0 ? -0.5 * (Bq + sq) : -0.5 * (Bq - sq);
            r1 = qq / A;
            r2 = qq != 0.0 ? Cq / qq : -1.0;
            if (r2 < r1) { double tt = r1; r1 = r2; r2 = tt; }
        }
    }
    if (r1 > 0.0 && r1 < 1.0) br[nb++] = r1;
    if (r2 > 0.0 && r2 < 1.0 && r2 != r1) br[nb++] = r2;
    br[nb] = 1.0;
    int n = 0;
    double ee = (double)(ex * ex + ey * ey);
    for (int j = 0; j < nb; j++) {
        double lo = br[j], hi = br[j + 1];
        double flo = cubic_at(F, lo), fhi = (j == nb - 1) ? f1 : cubic_at(F, hi);
        int slo = flo >= 0.0, shi = fhi >= 0.0;
        if (slo == shi) continue;
        for (int it = 0; it < 64; it++) {
            double mid = 0.5 * (lo + hi);
            if ((cubic_at(F, mid) >= 0.0) == slo) lo = mid; else hi = mid;
        }
        double t = 0.5 * (lo + hi);
        double sx = ((coef[6] * t + coef[4]) * t + coef[2]) * t + coef[0];
        double sy = ((coef[7] * t + coef[5]) * t + coef[3]) * t + coef[1];
        double q = ((sx - px) * ex + (sy - py) * ey) / ee;
        if (!(q >= 0.0 && q < 1.0)) continue;
        ts[n] = t; qs[n] = q; sg[n] = slo ? -1 : 1;
        n++;
    }
    return n;
}

/* [[p]] at spline parameter t of segment k (reading R27): G linear between
 * the markers, n and |dX/ds| from S'(t): [[p]] = dX (G x T) / |T|^2 with
 * G x T = G_x T_y - G_y T_x. */
static double spline_jump(const or_problem *p, const double *coef, const double *G, int k, double t)
{
    int kp = (k + 1) % p->n_markers;
    double Gx = (1.0 - t) * G[2 * k] + t * G[2 * kp], Gy = (1.0 - t) * G[2 * k + 1] + t * G[2 * kp + 1];
    double Tx = (3.0 * coef[6] * t + 2.0 * coef[4]) * t + coef[2];
    double Ty = (3.0 * coef[7] * t + 2.0 * coef[5]) * t + coef[3];
    return p->dX * (Gx * Ty - Gy * Tx) / (Tx * Tx + Ty * Ty);
}

/* ------------------------------------------------------------------------ */
/* Marker force and interface geometry.                                      */
/* ------------------------------------------------------------------------ */

/* G_k: spring membrane G = kappa (X_{k+1} - 2 X_k + X_{k-1}) / dX^2
 * (Sec. 2.2.2, Eq. (19)); rigid body direct forcing G = eta (U^D - U*) with
 * eta = 1/dt = 1 and U^D = 0 for a fixed body (Sec. 2.2.2, Eq. (18)).
 * n_k: outward unit normal (Sec. 3.1, Eq. (31); reading R7), rigid: radial.
 * J_k: |dX/ds| (reading R8), 1 for rigid bodies (Sec. 3.1).
 * jp_k = G.n / J = [[p]] (Sec. 3.1, Eq. (40)).
 * Gt_k = G - (G.n) n, the tangential part (Sec. 3.2, Eq. (46); reading R9). */
void or_marker_forces(const or_problem *p, const double *X, const double *U,
                      double *G, double *nrm, double *J, double *jp, double *Gt)
{
    int N = p->n_markers;
    double *Msp = NULL;
    if (p->interface == OR_IF_MEMBRANE && p->geometry == 1) {
        Msp = malloc(2 * N * sizeof(double));
        or_spline(p, X, Msp);
    }
    for (int k = 0; k < N; k++) {
        int km = (k + N - 1) % N, kp = (k + 1) % N;
        double gx, gy, nx_, ny_, jac;
        if (p->interface == OR_IF_MEMBRANE) {
            double d2 = p->dX * p->dX;
            gx = p->kappa * (X[2 * kp] - 2.0 * X[2 * k] + X[2 * km]) / d2;
            gy = p->kappa * (X[2 * kp + 1] - 2.0 * X[2 * k + 1] + X[2 * km + 1]) / d2;
            if (p->geometry == 1) {
                /* spline tangent at the knot, T = S_k'(0) (reading R27) */
                double tx = X[2 * kp] - X[2 * k] - (2.0 * Msp[2 * k] + Msp[2 * kp]) / 6.0;
                double ty = X[2 * kp + 1] - X[2 * k + 1] - (2.0 * Msp[2 * k + 1] + Msp[2 * kp + 1]) / 6.0;
                double tl = sqrt(tx * tx + ty * ty);
                nx_ = ty / tl;
                ny_ = -tx / tl;
                jac = tl / p->dX;
            } else {
                double tx = X[2 * kp] - X[2 * km], ty = X[2 * kp + 1] - X[2 * km + 1];
                double tl = sqrt(tx * tx + ty * ty);
                nx_ = ty / tl;
                ny_ = -tx / tl;
                double lp = hypot(X[2 * kp] - X[2 * k], X[2 * kp + 1] - X[2 * k + 1]);
                double lm = hypot(X[2 * k] - X[2 * km], X[2 * k + 1] - X[2 * km + 1]);
                jac = (lp + lm) / (2.0 * p->dX);
            }
        } else if (p->interface == OR_IF_NORMAL) {
            /* a uniform normal force G = F n on a fixed circle (Sec. 4.1) */
            nx_ = (X[2 * k] - p->cx) / p->radius;
            ny_ = (X[2 * k + 1] - p->cy) / p->radius;
            gx = p->f_normal * nx_;
            gy = p->f_normal * ny_;
            jac = 1.0;
        } else {
            double rx = X[2 * k] - p->cx, ry = X[2 * k + 1] - p->cy;
            gx = (p->ud[0] - p->ud[2] * ry) - U[2 * k];
            gy = (p->ud[1] + p->ud[2] * rx) - U[2 * k + 1];
            nx_ = rx / p->radius;
            ny_ = ry / p->radius;
            jac = 1.0;
        }
        double gn = gx * nx_ + gy * ny_;
        G[2 * k] = gx; G[2 * k + 1] = gy;
        nrm[2 * k] = nx_; nrm[2 * k + 1] = ny_;
        J[k] = jac;
        jp[k] = gn / jac;
        Gt[2 * k] = gx - gn * nx_;
        Gt[2 * k + 1] = gy - gn * ny_;
    }
    free(Msp);
}

/* ------------------------------------------------------------------------ */
/* Cut links (reading R10) and the jump of each population.                  */
/* ------------------------------------------------------------------------ */
#define SNAP 65536.0

static int64_t snap(double v) { return (int64_t)llrint(v * SNAP); }

/* (b - a) x (c - a), exact in 64-bit integers for |coordinates| < 2^29. */
static int64_t orient(int64_t ax, int64_t ay, int64_t bx, int64_t by, int64_t cx, int64_t cy)
{
    return (bx - ax) * (cy - ay) - (by - ay) * (cx - ax);
}

static int sgn64(int64_t v) { return (v > 0) - (v < 0); }

/* Side of the (perturbed) lattice node P + (eps, eps^2) w.r.t. the directed
 * chord A->B; never zero. */
static int side_of_node(int64_t ax, int64_t ay, int64_t bx, int64_t by, int64_t px, int64_t py)
{
    int64_t o = orient(ax, ay, bx, by, px, py);
    if (o != 0) return sgn64(o);
    if (by != ay) return -sgn64(by - ay);
    return sgn64(bx - ax);
}

/* Side of the chord end point A w.r.t. the perturbed link P->Q (same shift of
 * both link ends); never zero. */
static int side_of_marker(int64_t px, int64_t py, int64_t qx, int64_t qy, int64_t ax, int64_t ay)
{
    int64_t o = orient(px, py, qx, qy, ax, ay);
    if (o != 0) return sgn64(o);
    if (qy != py) return sgn64(qy - py);
    return -sgn64(qx - px);
}

/* Crossing test of link (x,y)->(x,y)+e_i with chord k of the snapped polygon.
 * Fills sigma (+1 interior->exterior, -1 reverse), q and theta on a hit. */
static int link_cuts_chord(int x, int y, int i, const int64_t *Ai, const int64_t *Bi,
                           int *sigma, double *q, double *theta)
{
    int64_t px = (int64_t)x * (int64_t)SNAP, py = (int64_t)y * (int64_t)SNAP;
    int64_t qx = (int64_t)(x + EX[i]) * (int64_t)SNAP, qy = (int64_t)(y + EY[i]) * (int64_t)SNAP;
    int sP = side_of_node(Ai[0], Ai[1], Bi[0], Bi[1], px, py);
    int sQ = side_of_node(Ai[0], Ai[1], Bi[0], Bi[1], qx, qy);
    if (sP == sQ) return 0;
    int sA = side_of_marker(px, py, qx, qy, Ai[0], Ai[1]);
    int sB = side_of_marker(px, py, qx, qy, Bi[0], Bi[1]);
    if (sA == sB) return 0;
    /* Counter-clockwise polygon: the interior lies to the left of A->B. */
    *sigma = (sP > 0) ? 1 : -1;
    double oP = (double)orient(Ai[0], Ai[1], Bi[0], Bi[1], px, py);
    double oQ = (double)orient(Ai[0], Ai[1], Bi[0], Bi[1], qx, qy);
    double oA = (double)orient(px, py, qx, qy, Ai[0], Ai[1]);
    double oB = (double)orient(px, py, qx, qy, Bi[0], Bi[1]);
    *q = oP / (oP - oQ);
    *theta = oA / (oA - oB);
    return 1;
}

/* Records every (link, chord) crossing of the closed snapped polygon, chord by
 * chord, testing the links whose source node lies within one lattice spacing
 * of the chord's bounding box (any crossing link has its source there). */
static int cutlinks_membrane(const or_problem *p, const double *X, const double *jp,
                             or_link *rec, int cap)
{
    int N = p->n_markers, n = 0;
    for (int k = 0; k < N; k++) {
        int kp = (k + 1) % N;
        int64_t A[2] = {snap(X[2 * k]), snap(X[2 * k + 1])};
        int64_t B[2] = {snap(X[2 * kp]), snap(X[2 * kp + 1])};
        double xmin = fmin(A[0], B[0]) / SNAP, xmax = fmax(A[0], B[0]) / SNAP;
        double ymin = fmin(A[1], B[1]) / SNAP, ymax = fmax(A[1], B[1]) / SNAP;
        for (int y = (int)floor(ymin) - 1; y <= (int)ceil(ymax) + 1; y++)
            for (int x = (int)floor(xmin) - 1; x <= (int)ceil(xmax) + 1; x++)
                for (int i = 1; i < 9; i++) {
                    int sg; double q, th;
                    if (!link_cuts_chord(x, y, i, A, B, &sg, &q, &th)) continue;
                    if (n < cap) {
                        or_link *r = &rec[n];
                        r->x = x; r->y = y; r->dir = i; r->sigma = sg; r->seg = k; r->pad = 0;
                        r->q = q; r->theta = th;
                        r->jp = (1.0 - th) * jp[k] + th * jp[kp];
                    }
                    n++;
                }
    }
    return n;
}

/* Every crossing of every link with the spline (reading R27), segment by
 * segment; the source nodes tested are those within one lattice spacing of
 * the bounding box of the segment's Bezier control points (the segment lies
 * in their hull).  theta is the spline parameter t of the crossing. */
int or_cutlinks_spline(const or_problem *p, const double *X, const double *G, or_link *rec, int cap)
{
    int N = p->n_markers, n = 0;
    double *M = malloc(2 * N * sizeof(double));
    or_spline(p, X, M);
    for (int k = 0; k < N; k++) {
        int kp = (k + 1) % N;
        double cf[8];
        spline_segment(N, X, M, k, cf);
        double hx[4], hy[4];
        hx[0] = cf[0]; hy[0] = cf[1];
        hx[1] = cf[0] + cf[2] / 3.0; hy[1] = cf[1] + cf[3] / 3.0;
        double t1x = cf[2] + 2.0 * cf[4] + 3.0 * cf[6], t1y = cf[3] + 2.0 * cf[5] + 3.0 * cf[7];
        hx[3] = X[2 * kp]; hy[3] = X[2 * kp + 1];
        hx[2] = hx[3] - t1x / 3.0; hy[2] = hy[3] - t1y / 3.0;
        double xmin = hx[0], xmax = hx[0], ymin = hy[0], ymax = hy[0];
        for (int j = 1; j < 4; j++) {
            xmin = fmin(xmin, hx[j]); xmax = fmax(xmax, hx[j]);
            ymin = fmin(ymin, hy[j]); ymax = fmax(ymax, hy[j]);
        }
        for (int y = (int)floor(ymin) - 1; y <= (int)ceil(ymax) + 1; y++)
            for (int x = (int)floor(xmin) - 1; x <= (int)ceil(xmax) + 1; x++)
                for (int i = 1; i < 9; i++) {
                    double ts[3], qs[3];
                    int sg[3];
                    int c = spline_link_crossings(cf, &X[2 * kp], x, y, EX[i], EY[i], ts, qs, sg);
                    for (int j = 0; j < c; j++) {
                        if (n < cap) {
                            or_link *r = &rec[n];
                            r->x = x; r->y = y; r->dir = i; r->sigma = sg[j]; r->seg = k; r->pad = 0;
                            r->q = qs[j]; r->theta = ts[j];
                            r->jp = spline_jump(p, cf, G, k, ts[j]);
                        }
                        n++;
                    }
                }
    }
    free(M);
    return n;
}

/* Rigid circle: level set phi(x) = |x - c|^2 - R^2 (Sec. 3.2 uses a level set
 * for rigid bodies); phi < 0 is the interior.  With integer centre and radius
 * phi is exact.  [[p]] at the cut point is linear in angle between the two
 * markers that bracket it (markers at angles 2 pi k / N). */
static double circle_phi(const or_problem *p, double x, double y)
{
    return (x - p->cx) * (x - p->cx) + (y - p->cy) * (y - p->cy) - p->radius * p->radius;
}

static int cutlinks_rigid(const or_problem *p, const double *jp, or_link *rec, int cap)
{
    int N = p->n_markers, n = 0;
    int x0 = (int)floor(p->cx - p->radius) - 2, x1 = (int)ceil(p->cx + p->radius) + 2;
    int y0 = (int)floor(p->cy - p->radius) - 2, y1 = (int)ceil(p->cy + p->radius) + 2;
    for (int y = y0; y <= y1; y++)
        for (int x = x0; x <= x1; x++)
            for (int i = 1; i < 9; i++) {
                int inP = circle_phi(p, x, y) < 0.0;
                int inQ = circle_phi(p, x + EX[i], y + EY[i]) < 0.0;
                if (inP == inQ) continue;
                /* |P + q e - c|^2 = R^2 */
                double dx = x - p->cx, dy = y - p->cy;
                double ee = EX[i] * EX[i] + EY[i] * EY[i];
                double de = dx * EX[i] + dy * EY[i];
                double dd = dx * dx + dy * dy - p->radius * p->radius;
                double disc = sqrt(de * de - ee * dd);
                double q = inP ? (-de + disc) / ee : (-de - disc) / ee;
                double cxp = x + q * EX[i] - p->cx, cyp = y + q * EY[i] - p->cy;
                double ang = atan2(cyp, cxp) - p->theta;   /* theta in [0, 2 pi) */
                if (ang < 0.0) ang += 2.0 * M_PI;
                if (ang < 0.0) ang += 2.0 * M_PI;
                if (ang >= 2.0 * M_PI) ang -= 2.0 * M_PI;
                double s = ang * N / (2.0 * M_PI);
                int k = (int)floor(s);
                if (k >= N) k = N - 1;
                double t = s - k;
                int kp = (k + 1) % N;
                if (n < cap) {
                    or_link *r = &rec[n];
                    r->x = x; r->y = y; r->dir = i; r->sigma = inP ? 1 : -1; r->seg = k; r->pad = 0;
                    r->q = q; r->theta = t;
                    r->jp = (1.0 - t) * jp[k] + t * jp[kp];
                }
                n++;
            }
    return n;
}

int or_cutlinks(const or_problem *p, const double *X, const double *jp, or_link *rec, int cap)
{
    if (p->interface == OR_IF_MEMBRANE) return cutlinks_membrane(p, X, jp, rec, cap);
    if (p->interface == OR_IF_RIGID || p->interface == OR_IF_NORMAL) return cutlinks_rigid(p, jp, rec, cap);
    return 0;
}

/* Brute force over every link of the box [x0,x1]x[y0,y1] and every chord; the
 * independent check of the chord-by-chord enumeration above. */
int or_cutlinks_bruteforce(const or_problem *p, const double *X, const double *jp,
                           int x0, int x1, int y0, int y1, or_link *rec, int cap)
{
    int N = p->n_markers, n = 0;
    for (int k = 0; k < N; k++) {
        int kp = (k + 1) % N;
        int64_t A[2] = {snap(X[2 * k]), snap(X[2 * k + 1])};
        int64_t B[2] = {snap(X[2 * kp]), snap(X[2 * kp + 1])};
        for (int y = y0; y <= y1; y++)
            for (int x = x0; x <= x1; x++)
                for (int i = 1; i < 9; i++) {
                    int sg; double q, th;
                    if (!link_cuts_chord(x, y, i, A, B, &sg, &q, &th)) continue;
                    if (n < cap) {
                        or_link *r = &rec[n];
                        r->x = x; r->y = y; r->dir = i; r->sigma = sg; r->seg = k; r->pad = 0;
                        r->q = q; r->theta = th;
                        r->jp = (1.0 - th) * jp[k] + th * jp[kp];
                    }
                    n++;
                }
    }
    return n;
}

/* Point-in-polygon of a (perturbed) node by counting chord crossings of the
 * ray from the node in +x, with the same snapped chords and tie rule as the
 * link test: used only by tests to relate crossings to inside/outside. */
int or_node_inside(const or_problem *p, const double *X, int x, int y)
{
    int N = p->n_markers, c = 0;
    for (int k = 0; k < N; k++) {
        int kp = (k + 1) % N;
        int64_t A[2] = {snap(X[2 * k]), snap(X[2 * k + 1])};
        int64_t B[2] = {snap(X[2 * kp]), snap(X[2 * kp + 1])};
        /* ray = straight path from (x,y) to (nx + 8, y), beyond every marker */
        int64_t px = (int64_t)x * (int64_t)SNAP, py = (int64_t)y * (int64_t)SNAP;
        int64_t qx = (int64_t)(p->nx + 8) * (int64_t)SNAP, qy = py;
        int sP = side_of_node(A[0], A[1], B[0], B[1], px, py);
        int sQ = side_of_node(A[0], A[1], B[0], B[1], qx, qy);
        if (sP == sQ) continue;
        int sA = side_of_marker(px, py, qx, qy, A[0], A[1]);
        int sB = side_of_marker(px, py, qx, qy, B[0], B[1]);
        if (sA == sB) continue;
        c ^= 1;
    }
    return c;
}

/* ------------------------------------------------------------------------ */
/* Boundaries: non-equilibrium extrapolation (reading R12).                  */
/* ------------------------------------------------------------------------ */
static void nee_node(const or_problem *p, double *f, int x, int y)
{
    int inx = 0, iny = 0;
    if (p->bc[0] != OR_PERIODIC && x == 0) inx = 1;
    if (p->bc[1] != OR_PERIODIC && x == p->nx - 1) inx = -1;
    if (p->bc[2] != OR_PERIODIC && y == 0) iny = 1;
    if (p->bc[3] != OR_PERIODIC && y == p->ny - 1) iny = -1;
    if (inx == 0 && iny == 0) return;
    int xf = x + inx, yf = y + iny;
    double ff[9], rf, uxf, uyf;
    for (int i = 0; i < 9; i++) ff[i] = f[idx(p, i, xf, yf)];
    or_moments_node(ff, &rf, &uxf, &uyf);
    double ubx = 0.0, uby = 0.0;
    int side_type;
    if (iny != 0) {
        /* y side (corners included) follows its wall rule */
        int s = (iny > 0) ? 2 : 3;
        side_type = p->bc[s];
        if (side_type == OR_WALL) { ubx = p->u_wall[s]; uby = 0.0; }
    } else {
        int s = (inx > 0) ? 0 : 1;
        side_type = p->bc[s];
        if (side_type == OR_WALL) { ubx = 0.0; uby = p->u_wall[s]; }
    }
    if (side_type == OR_INLET) {
        double H = p->ny - 1;
        ubx = 4.0 * p->u_max * y * (H - y) / (H * H);
        uby = 0.0;
    } else if (side_type == OR_INLET_UNIFORM) {
        ubx = p->u_max;
        uby = 0.0;
    } else if (side_type == OR_OUTLET) {
        ubx = uxf; uby = uyf;
    }
    double eb[9], ef[9];
    or_equilibrium(rf, ubx, uby, eb);
    or_equilibrium(rf, uxf, uyf, ef);
    for (int i = 0; i < 9; i++) f[idx(p, i, x, y)] = eb[i] + (ff[i] - ef[i]);
}

void or_boundaries(const or_problem *p, double *f)
{
    for (int y = 0; y < p->ny; y++)
        for (int x = 0; x < p->nx; x++) {
            int edge = (x == 0 || x == p->nx - 1 || y == 0 || y == p->ny - 1);
            if (edge) nee_node(p, f, x, y);
        }
}

/* ------------------------------------------------------------------------ */
/* One time step.                                                            */
/* ------------------------------------------------------------------------ */
typedef struct {
    double *U, *G, *nrm, *J, *jp, *Gt;   /* [2N], [2N], [2N], [N], [N], [2N] */
    double *gx, *gy;                     /* spread force planes [ny*nx] */
    or_link *links; int links_cap; int n_links;
} or_step_out;

/* One II-LBM step, Sec. 3.2 Eq. (47):
 *   f_i(x, n+1) = f*_i(x - e_i, n) + sigma [[f_i]] + (force already in f*),
 * with [[f_i]] = w_i [[p]] / c_s^2 (Sec. 3.1, Eq. (32)) on every cut link,
 * f* = collide(f) + w_i e_i.g_par / c_s^2, g_par the spread tangential force;
 * then X^{n+1} = X^n + U^n (Sec. 2.2.2, Eq. (20)).
 * Under the IB-LBM force modes the full G is spread and no jump is applied
 * (Sec. 2.2.2, Eq. (16)-(17)), the comparison method of the paper, and a
 * membrane then moves with the velocity its distributions carry after this
 * step's force (reading R18); the Guo modes collide with Guo's term of the
 * spread force (reading R24). */
int or_step(const or_problem *p, double *f, double *X, or_step_out *out)
{
    int nx = p->nx, ny = p->ny, N = p->n_markers;
    long nn = (long)nx * ny;
    double *rho = calloc(nn, sizeof(double)), *ux = calloc(nn, sizeof(double)), *uy = calloc(nn, sizeof(double));
    double *gx = calloc(nn, sizeof(double)), *gy = calloc(nn, sizeof(double));
    double *fpost = calloc(9 * nn, sizeof(double)), *jump = calloc(9 * nn, sizeof(double));
    double *U = calloc(2 * N + 2, sizeof(double)), *G = calloc(2 * N + 2, sizeof(double));
    double *nrm = calloc(2 * N + 2, sizeof(double)), *J = calloc(N + 1, sizeof(double));
    double *jp = calloc(N + 1, sizeof(double)), *Gt = calloc(2 * N + 2, sizeof(double));
    int nl = 0, bad = 0;
    or_link *links = NULL;
    double M[81], Minv[81];
    or_mrt_matrices(M, Minv);

    /* 0. the bounded-side nodes of f^n obey the extrapolation rule; it only
     *    reads interior nodes and is idempotent, so this changes nothing
     *    after the first step and makes any initial state consistent */
    or_boundaries(p, f);
    /* 1. moments of f^n; uniform body force */
    or_moments(p, f, rho, ux, uy);
    for (long n = 0; n < nn; n++) { gx[n] = p->body[0]; gy[n] = p->body[1]; }
    /* under Guo's term the velocity carries half the force (reading R24);
     * before the spread that is the body force alone */
    double *jx = NULL, *jy = NULL;
    if (uses_guo(p)) {
        jx = calloc(nn, sizeof(double)); jy = calloc(nn, sizeof(double));
        memcpy(jx, ux, nn * sizeof(double)); memcpy(jy, uy, nn * sizeof(double));
        for (long n = 0; n < nn; n++) {
            ux[n] = (jx[n] + 0.5 * gx[n]) / rho[n];
            uy[n] = (jy[n] + 0.5 * gy[n]) / rho[n];
        }
    }

    if (p->interface != OR_IF_NONE && N > 0) {
        /* 2. marker velocity from u^n; force, normal, [[p]], tangential part */
        or_interp(p, ux, uy, X, U);
        or_marker_forces(p, X, U, G, nrm, J, jp, Gt);
        /* 3. spread the tangential force (the full force under IB-LBM) */
        or_spread(p, X, has_jumps(p) ? Gt : G, gx, gy);
        /* 3b. the velocity a membrane moves with, now that the whole force g
         *     of this step is known (a membrane's force depends on X alone):
         *     - II-LBM with Guo's term: u = (j + g/2) / rho (Sec. 2.2.2);
         *     - the IB-LBM comparison modes (reading R18): each scheme's own
         *       velocity taken from the distributions after this step's
         *       collision and force term, whose momentum is j + g: the simple
         *       term's u = j + g, Guo's u = (j + g + g/2) / rho */
        if (p->interface == OR_IF_MEMBRANE && (uses_guo(p) || !has_jumps(p))) {
            double c = has_jumps(p) ? 0.5 : (uses_guo(p) ? 1.5 : 1.0);
            for (long n = 0; n < nn; n++) {
                double j0 = uses_guo(p) ? jx[n] : ux[n], j1 = uses_guo(p) ? jy[n] : uy[n];
                double r = uses_guo(p) ? rho[n] : 1.0;
                ux[n] = (j0 + c * gx[n]) / r;
                uy[n] = (j1 + c * gy[n]) / r;
            }
            or_interp(p, ux, uy, X, U);
        }
        /* 4. cut links and the per-link jump sigma w_i [[p]] / c_s^2 */
        if (has_jumps(p)) {
            int cap = 64 * N + 4096;
            links = calloc(cap, sizeof(or_link));
            if (p->interface == OR_IF_MEMBRANE && p->geometry == 1)
                nl = or_cutlinks_spline(p, X, G, links, cap);
            else
                nl = or_cutlinks(p, X, jp, links, cap);
            if (nl > cap) nl = cap;
            for (int l = 0; l < nl; l++) {
                const or_link *r = &links[l];
                int xs = wrap_x(p, r->x), ys = wrap_y(p, r->y);
                if (xs < 0 || ys < 0) { bad = 1; continue; }
                jump[idx(p, r->dir, xs, ys)] += r->sigma * WT[r->dir] * r->jp / CS2;
            }
        }
    }

    /* 5. collide at every node with the force term */
#pragma omp parallel for
    for (int y = 0; y < ny; y++)
        for (int x = 0; x < nx; x++) {
            double fn[9], fo[9];
            long n = (long)y * nx + x;
            for (int i = 0; i < 9; i++) fn[i] = f[idx(p, i, x, y)];
            if (uses_guo(p))
                collide_guo(p, M, Minv, fn, gx[n], gy[n], fo);
            else
                collide_with(p, M, Minv, fn, gx[n], gy[n], fo);
            for (int i = 0; i < 9; i++) fpost[idx(p, i, x, y)] = fo[i];
        }

    /* 6. stream with the jump of every cut link (source node x - e_i) */
#pragma omp parallel for collapse(2)
    for (int i = 0; i < 9; i++)
        for (int y = 0; y < ny; y++)
            for (int x = 0; x < nx; x++) {
                int xs = wrap_x(p, x - EX[i]), ys = wrap_y(p, y - EY[i]);
                if (xs < 0 || ys < 0) { f[idx(p, i, x, y)] = NAN; continue; }
                f[idx(p, i, x, y)] = fpost[idx(p, i, xs, ys)] + jump[idx(p, i, xs, ys)];
            }

    /* 7. outer boundaries */
    or_boundaries(p, f);

    /* 8. marker update X^{n+1} = X^n + U^n (a fixed rigid body stays put) */
    if (p->interface == OR_IF_MEMBRANE)
        for (int k = 0; k < 2 * N; k++) X[k] += U[k];

    if (out) {
        if (out->U) memcpy(out->U, U, 2 * N * sizeof(double));
        if (out->G) memcpy(out->G, G, 2 * N * sizeof(double));
        if (out->nrm) memcpy(out->nrm, nrm, 2 * N * sizeof(double));
        if (out->J) memcpy(out->J, J, N * sizeof(double));
        if (out->jp) memcpy(out->jp, jp, N * sizeof(double));
        if (out->Gt) memcpy(out->Gt, Gt, 2 * N * sizeof(double));
        if (out->gx) memcpy(out->gx, gx, nn * sizeof(double));
        if (out->gy) memcpy(out->gy, gy, nn * sizeof(double));
        if (out->links) {
            int m = nl < out->links_cap ? nl : out->links_cap;
            if (m > 0) memcpy(out->links, links, m * sizeof(or_link));
        }
        out->n_links = nl;
    }
    free(rho); free(ux); free(uy); free(gx); free(gy); free(fpost); free(jump);
    free(U); free(G); free(nrm); free(J); free(jp); free(Gt); free(links); free(jx); free(jy);
    return bad ? -1 : 0;
}

/* Runs n_steps; optional per-step force on the body F = -sum_k G_k dX
 * (Sec. 2.3, Eq. (25) without the interior-inertia term, fixed body). */
int or_run(const or_problem *p, double *f, double *X, int n_steps, double *force_hist)
{
    int N = p->n_markers;
    double *G = calloc(2 * N + 2, sizeof(double));
    or_step_out o;
    memset(&o, 0, sizeof o);
    o.G = G;
    int rc = 0;
    for (int s = 0; s < n_steps && rc == 0; s++) {
        rc = or_step(p, f, X, &o);
        if (force_hist) {
            double fx = 0.0, fy = 0.0;
            for (int k = 0; k < N; k++) { fx -= G[2 * k] * p->dX; fy -= G[2 * k + 1] * p->dX; }
            force_hist[2 * s] = fx; force_hist[2 * s + 1] = fy;
        }
    }
    free(G);
    return rc;
}

/* ------------------------------------------------------------------------ */
/* Rigid-body dynamics of a circle (Sec. 2.3).                               */
/* ------------------------------------------------------------------------ */
typedef struct {
    int32_t free_dofs;     /* bit 0: x, bit 1: y, bit 2: rotation */
    int32_t pad;
    double rho_star;       /* rho_s / rho_f */
    double spring[2];      /* k_s per axis, about the initial centre */
    double damping[2];     /* c per axis */
    double presc_amp[2];   /* prescribed harmonic motion D_c = -A sin(U_max t / A) ... */
    double presc_umax[2];  /* ... U_c = -U_max cos(U_max t / A) (Sec. 4.4); 0: none */
} or_body_params;

typedef struct {
    double c[2], U[2], a[2];   /* centre, velocity, acceleration of the centre */
    double theta, W, wdot;     /* orientation, angular velocity and acceleration */
    double Uprev[2], Wprev;    /* the previous step's velocities (interior inertia) */
    double F[2], T;            /* F^ext and T^ext of the last step */
    double c0[2];              /* initial centre */
    int64_t n;                 /* steps taken */
} or_body;

/* One step with a moving circle:
 *  - the prescribed axes take U_c(n) and X_c(n) from the harmonic motion;
 *  - the step runs with U^D = U_c + W x (X - X_c) at the markers (Sec. 2.2.2, Eq. (18));
 *  - F^ext = -sum G dX + rho_f V_s (U_c^n - U_c^{n-1}) and
 *    T^ext = -sum (X - X_c) x G dX + (rho_f/rho_s) I_s (W^n - W^{n-1})
 *    (Sec. 2.3, the total force and torque; rho_f = 1, V_s = pi R^2,
 *    m = rho_s V_s, I_s = m R^2 / 2), plus spring and damper on free axes;
 *  - m a^{n+1} = F, I_s w^{n+1} = T; U^{n+1} = U^n + a^{n+1};
 *    X_c^{n+1} = X_c^n + U^n + (a^n + a^{n+1}) / 2, the same for theta;
 *  - the markers are placed rigidly: X_k = X_c + R (cos, sin)(theta + 2 pi k / N). */
int or_step_body(const or_problem *p0, const or_body_params *bp, or_body *b, double *f, double *X)
{
    int N = p0->n_markers;
    double t = (double)b->n;
    for (int ax = 0; ax < 2; ax++)
        if (bp->presc_umax[ax] != 0.0) {
            double A = bp->presc_amp[ax], Um = bp->presc_umax[ax];
            b->U[ax] = -Um * cos(Um * t / A);
            b->c[ax] = b->c0[ax] - A * sin(Um * t / A);
        }
    if (b->n == 0) {
        b->Uprev[0] = b->U[0]; b->Uprev[1] = b->U[1]; b->Wprev = b->W;
    }
    for (int k = 0; k < N; k++) {
        double ang = b->theta + 2.0 * M_PI * k / N;
        X[2 * k] = b->c[0] + p0->radius * cos(ang);
        X[2 * k + 1] = b->c[1] + p0->radius * sin(ang);
    }
    or_problem p = *p0;
    p.cx = b->c[0]; p.cy = b->c[1];
    p.ud[0] = b->U[0]; p.ud[1] = b->U[1]; p.ud[2] = b->W;
    p.theta = b->theta - 2.0 * M_PI * floor(b->theta / (2.0 * M_PI));
    double *G = calloc(2 * N + 2, sizeof(double));
    or_step_out o;
    memset(&o, 0, sizeof o);
    o.G = G;
    int rc = or_step(&p, f, X, &o);
    double R = p0->radius, Vs = M_PI * R * R;
    double m = bp->rho_star * Vs, Is = 0.5 * m * R * R;
    double Fx = 0.0, Fy = 0.0, T = 0.0;
    for (int k = 0; k < N; k++) {
        double rx = X[2 * k] - b->c[0], ry = X[2 * k + 1] - b->c[1];
        Fx -= G[2 * k] * p0->dX;
        Fy -= G[2 * k + 1] * p0->dX;
        T -= (rx * G[2 * k + 1] - ry * G[2 * k]) * p0->dX;
    }
    Fx += Vs * (b->U[0] - b->Uprev[0]);
    Fy += Vs * (b->U[1] - b->Uprev[1]);
    T += Is / bp->rho_star * (b->W - b->Wprev);
    b->F[0] = Fx; b->F[1] = Fy; b->T = T;
    double Fa[2] = {Fx, Fy};
    double Unew[2] = {b->U[0], b->U[1]};
    for (int ax = 0; ax < 2; ax++) {
        b->Uprev[ax] = b->U[ax];
        if (bp->presc_umax[ax] != 0.0) {
            /* the state left for the next step, as on a free axis */
            double A = bp->presc_amp[ax], Um = bp->presc_umax[ax];
            Unew[ax] = -Um * cos(Um * (t + 1.0) / A);
            b->c[ax] = b->c0[ax] - A * sin(Um * (t + 1.0) / A);
            continue;
        }
        if (!(bp->free_dofs & (1 << ax))) continue;
        double Fext = Fa[ax] - bp->spring[ax] * (b->c[ax] - b->c0[ax]) - bp->damping[ax] * b->U[ax];
        double anew = Fext / m;
        Unew[ax] = b->U[ax] + anew;
        b->c[ax] = b->c[ax] + b->U[ax] + 0.5 * (b->a[ax] + anew);
        b->a[ax] = anew;
    }
    b->U[0] = Unew[0]; b->U[1] = Unew[1];
    b->Wprev = b->W;
    if (bp->free_dofs & 4) {
        double wnew = T / Is;
        double Wn = b->W + wnew;
        b->theta = b->theta + b->W + 0.5 * (b->wdot + wnew);
        b->wdot = wnew;
        b->W = Wn;
    }
    b->n++;
    /* markers of the next step */
    for (int k = 0; k < N; k++) {
        double ang = b->theta + 2.0 * M_PI * k / N;
        X[2 * k] = b->c[0] + p0->radius * cos(ang);
        X[2 * k + 1] = b->c[1] + p0->radius * sin(ang);
    }
    free(G);
    return rc;
}

int or_sizeof_body(void) { return (int)sizeof(or_body); }
int or_sizeof_body_params(void) { return (int)sizeof(or_body_params); }

/* ------------------------------------------------------------------------ */
/* Diagnostics.                                                              */
/* ------------------------------------------------------------------------ */

/* Enclosed area of the marker polygon (shoelace formula). */
double or_polygon_area(int N, const double *X)
{
    double a = 0.0;
    for (int k = 0; k < N; k++) {
        int kp = (k + 1) % N;
        a += X[2 * k] * X[2 * kp + 1] - X[2 * kp] * X[2 * k + 1];
    }
    return 0.5 * a;
}

static double seg_dist(double px, double py, double ax, double ay, double bx, double by)
{
    double vx = bx - ax, vy = by - ay, wx = px - ax, wy = py - ay;
    double t = (vx * wx + vy * wy) / (vx * vx + vy * vy);
    if (t < 0.0) t = 0.0;
    if (t > 1.0) t = 1.0;
    double dx = px - (ax + t * vx), dy = py - (ay + t * vy);
    return sqrt(dx * dx + dy * dy);
}

/* Mean pressure p = c_s^2 rho over interior nodes farther than `margin` from
 * the polygon minus the same over exterior nodes (uses the rho field). */
double or_pressure_jump(const or_problem *p, const double *rho, const double *X, double margin)
{
    int N = p->n_markers;
    double sin_ = 0.0, sout = 0.0;
    long cin = 0, cout = 0;
    for (int y = 0; y < p->ny; y++)
        for (int x = 0; x < p->nx; x++) {
            double d = 1e300;
            for (int k = 0; k < N; k++) {
                int kp = (k + 1) % N;
                double dd = seg_dist(x, y, X[2 * k], X[2 * k + 1], X[2 * kp], X[2 * kp + 1]);
                if (dd < d) d = dd;
            }
            if (d < margin) continue;
            double pr = CS2 * rho[(long)y * p->nx + x];
            if (or_node_inside(p, X, x, y)) { sin_ += pr; cin++; } else { sout += pr; cout++; }
        }
    if (cin == 0 || cout == 0) return NAN;
    return sin_ / cin - sout / cout;
}

int or_sizeof_link(void) { return (int)sizeof(or_link); }

/* Threads the OpenMP loops of the oracle use (1 without OpenMP). */
#ifdef _OPENMP
#include <omp.h>
int or_num_threads(void) { return omp_get_max_threads(); }
void or_set_num_threads(int n) { if (n > 0) omp_set_num_threads(n); }
#else
int or_num_threads(void) { return 1; }
void or_set_num_threads(int n) { (void)n; }
#endif
int or_sizeof_problem(void) { return (int)sizeof(or_problem); }
