// D3Q19 form of the II-LBM on one MI355X: a periodic box, SRT or MRT with the
// He-Luo equilibrium and the simple force term, and one immersed surface:
//   - a fixed sphere with a uniform normal force, entered as jumps on the links
//     its level set cuts (II-LBM) or as a force field spread from surface
//     markers (IB-LBM);
//   - a fixed closed triangulation with vertex jumps (exact link search once,
//     jumps applied after every sweep);
//   - a deformable triangulated membrane under surface tension (II-LBM or
//     IB-LBM), a fixed rigid triangulated surface held by direct forcing, or a
//     free rigid sphere; these find their links again every step.
//
// Storage: FP32 deviations d_i = f_i - w_i, planes [19][nz][ny][pitch].  The
// sweep pulls d_i from x - e_i, collides, adds the force term and (II-LBM) the
// jumps of the links this node sends, and stores once at x, so the next pull
// reads f^{n+1}_i(x + e_i) with its jump already in place.  The triangulated
// surfaces add their jumps to the stored populations of the sending nodes
// after the sweep, to the same effect.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <vector>

#include "../../include/ii_lbm3.h"

namespace iilbm3 {

constexpr int kQ = 19;
constexpr int E3X[kQ] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0};
constexpr int E3Y[kQ] = {0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, 1, -1};
constexpr int E3Z[kQ] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1};
constexpr double W3D[kQ] = {1.0 / 3.0, 1.0 / 18.0, 1.0 / 18.0, 1.0 / 18.0, 1.0 / 18.0, 1.0 / 18.0,
                            1.0 / 18.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0,
                            1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0,
                            1.0 / 36.0};
constexpr int kBX = 256;

// The orthogonal 19-moment basis of d'Humieres et al. (2002), the 3-D form of
// the Lallemand-Luo basis behind the paper's MRT (Sec. 2.2.1): row k is a
// polynomial in the velocity (cx, cy, cz), evaluated at compile time so the
// unrolled transforms keep only the non-zero integer coefficients.
constexpr int basis_row(int k, int x, int y, int z)
{
    const int c2 = x * x + y * y + z * z;
    switch (k) {
    case 0: return 1;
    case 1: return 19 * c2 - 30;
    case 2: return (21 * c2 * c2 - 53 * c2 + 24) / 2;
    case 3: return x;
    case 4: return (5 * c2 - 9) * x;
    case 5: return y;
    case 6: return (5 * c2 - 9) * y;
    case 7: return z;
    case 8: return (5 * c2 - 9) * z;
    case 9: return 3 * x * x - c2;
    case 10: return (3 * c2 - 5) * (3 * x * x - c2);
    case 11: return y * y - z * z;
    case 12: return (3 * c2 - 5) * (y * y - z * z);
    case 13: return x * y;
    case 14: return y * z;
    case 15: return x * z;
    case 16: return x * (y * y - z * z);
    case 17: return y * (z * z - x * x);
    default: return z * (x * x - y * y);
    }
}

struct Basis3 {
    int m[kQ][kQ];
};

constexpr Basis3 make_basis3()
{
    Basis3 b{};
    for (int k = 0; k < kQ; k++)
        for (int i = 0; i < kQ; i++) b.m[k][i] = basis_row(k, E3X[i], E3Y[i], E3Z[i]);
    return b;
}

constexpr Basis3 kM3 = make_basis3();

// Rows odd in the velocity: j, q and the third-order m.
constexpr bool kOddRow[kQ] = {false, false, false, true, true, true, true, true, true, false,
                              false, false, false, false, false, false, true, true, true};

// Populations 2p - 1 and 2p are opposite, and each row is even or odd.
constexpr bool check_pairs()
{
    for (int p = 1; p < 10; p++) {
        if (E3X[2 * p - 1] != -E3X[2 * p] || E3Y[2 * p - 1] != -E3Y[2 * p] || E3Z[2 * p - 1] != -E3Z[2 * p])
            return false;
        for (int k = 0; k < kQ; k++)
            if (kM3.m[k][2 * p - 1] != (kOddRow[k] ? -kM3.m[k][2 * p] : kM3.m[k][2 * p])) return false;
    }
    for (int k = 0; k < kQ; k++)
        if (kOddRow[k] && kM3.m[k][0] != 0) return false;
    return true;
}
static_assert(check_pairs(), "opposite populations and row parity");

struct Box {
    int nx, ny, nz, pitch;
    long long plane;        // elements per population (pitch * ny * nz)
    double omega;
    double g[3];            // body force
    int sphere, ib;
    double cx, cy, cz, R, F;
    double sk[kQ];          // MRT: rate of moment k over the squared norm of its row
};

__device__ __forceinline__ int wrapi(int v, int n) { return v < 0 ? v + n : (v >= n ? v - n : v); }

// Level set of the sphere, |x - c|^2 - R^2 (interior < 0), in FP64.
__device__ __forceinline__ double sphere_phi(const Box& b, double x, double y, double z)
{
    const double dx = x - b.cx, dy = y - b.cy, dz = z - b.cz;
    return dx * dx + dy * dy + dz * dz - b.R * b.R;
}

// The spread force field is summed in 64-bit fixed point at 2^-56 (terms
// clamped to 64 in magnitude), so that it is exact and does not depend on
// the order in which the threads add their terms.
constexpr double kFix3 = 72057594037927936.0;   // 2^56

__device__ __forceinline__ long long fix3(double v)
{
    const double c = isfinite(v) ? fmin(fmax(v, -64.0), 64.0) : 64.0;
    return __double2ll_rn(c * kFix3);
}

__device__ __forceinline__ void fix3_add(long long* p, double v)
{
    atomicAdd((unsigned long long*)p, (unsigned long long)fix3(v));
}

__device__ __forceinline__ double fix3_get(long long q) { return (double)q * (1.0 / kFix3); }

template <bool IB, bool MRT>
__global__ __launch_bounds__(kBX) void k_sweep3(Box b, const float* __restrict__ A,
                                                float* __restrict__ B,
                                                const long long* __restrict__ gfield)
{
    const int x = blockIdx.x * kBX + threadIdx.x;
    const int y = blockIdx.y, z = blockIdx.z;
    if (x >= b.nx) return;
    const long long row = ((long long)z * b.ny + y) * b.pitch;
    double d[kQ];
#pragma unroll
    for (int i = 0; i < kQ; i++) {
        const int xs = wrapi(x - E3X[i], b.nx), ys = wrapi(y - E3Y[i], b.ny), zs = wrapi(z - E3Z[i], b.nz);
        d[i] = (double)A[i * b.plane + ((long long)zs * b.ny + ys) * b.pitch + xs];
    }
    // moments of the deviations: rho - 1 and j = sum e d
    double r = 0.0, jx = 0.0, jy = 0.0, jz = 0.0;
#pragma unroll
    for (int i = 0; i < kQ; i++) {
        r += d[i];
        jx += E3X[i] * d[i];
        jy += E3Y[i] * d[i];
        jz += E3Z[i] * d[i];
    }
    double gx = b.g[0], gy = b.g[1], gz = b.g[2];
    if (IB) {
        const long long c = ((long long)z * b.ny + y) * b.nx + x;
        const long long n = (long long)b.nx * b.ny * b.nz;
        gx += fix3_get(gfield[c]);
        gy += fix3_get(gfield[n + c]);
        gz += fix3_get(gfield[2 * n + c]);
    }
    const double jj = jx * jx + jy * jy + jz * jz;
    // He-Luo equilibrium deviation w_i [dr + 3 e.j + 4.5 (e.j)^2 - 1.5 j.j],
    // SRT or MRT relaxation and the force term 3 w_i e.g
    if (MRT) {
        // m - m_eq = M (f - f_eq); f* = f - M^T diag(s_k / |row k|^2) (m - m_eq);
        // rho and j (rows 0, 3, 5, 7) are conserved and skipped.  Populations
        // 2p-1 and 2p are opposite (p = 1..9), and every row is even or odd in
        // the velocity, so even rows see only the pair sums, odd rows only the
        // pair differences, and the update of a pair is (E + O, E - O).
        double dev[kQ];
#pragma unroll
        for (int i = 0; i < kQ; i++) {
            const double ej = E3X[i] * jx + E3Y[i] * jy + E3Z[i] * jz;
            dev[i] = d[i] - W3D[i] * (r + 3.0 * ej + 4.5 * ej * ej - 1.5 * jj);
        }
        double sp[10], dp[10];            // pair sums / differences; sp[0] = rest
        sp[0] = dev[0];
        dp[0] = 0.0;
#pragma unroll
        for (int q = 1; q < 10; q++) {
            sp[q] = dev[2 * q - 1] + dev[2 * q];
            dp[q] = dev[2 * q - 1] - dev[2 * q];
        }
        double m[kQ];
#pragma unroll
        for (int k = 0; k < kQ; k++) {
            m[k] = 0.0;
            if (k == 0 || k == 3 || k == 5 || k == 7) continue;
            const bool odd = kOddRow[k];
            if (!odd && kM3.m[k][0] != 0) m[k] += kM3.m[k][0] * sp[0];
#pragma unroll
            for (int q = 1; q < 10; q++)
                if (kM3.m[k][2 * q - 1] != 0) m[k] += kM3.m[k][2 * q - 1] * (odd ? dp[q] : sp[q]);
            m[k] *= b.sk[k];
        }
        double ev[10], od[10];
#pragma unroll
        for (int q = 0; q < 10; q++) {
            const int i = q == 0 ? 0 : 2 * q - 1;
            ev[q] = 0.0;
            od[q] = 0.0;
#pragma unroll
            for (int k = 0; k < kQ; k++) {
                if (k == 0 || k == 3 || k == 5 || k == 7 || kM3.m[k][i] == 0) continue;
                if (kOddRow[k]) od[q] += kM3.m[k][i] * m[k];
                else ev[q] += kM3.m[k][i] * m[k];
            }
        }
#pragma unroll
        for (int i = 0; i < kQ; i++) {
            const int q = (i + 1) / 2;
            const double a = i == 0 ? ev[0] : ((i & 1) ? ev[q] + od[q] : ev[q] - od[q]);
            const double eg = E3X[i] * gx + E3Y[i] * gy + E3Z[i] * gz;
            d[i] = d[i] - a + 3.0 * W3D[i] * eg;
        }
    } else {
#pragma unroll
        for (int i = 0; i < kQ; i++) {
            const double ej = E3X[i] * jx + E3Y[i] * jy + E3Z[i] * jz;
            const double eg = E3X[i] * gx + E3Y[i] * gy + E3Z[i] * gz;
            const double deq = W3D[i] * (r + 3.0 * ej + 4.5 * ej * ej - 1.5 * jj);
            d[i] = d[i] + b.omega * (deq - d[i]) + 3.0 * W3D[i] * eg;
        }
    }
    if (!IB && b.sphere) {
        // jumps of the links this node sends (Sec. 3.1, Eq. (32)): only a node
        // within sqrt 2 of the sphere can send a cut link
        const double ph = sphere_phi(b, x, y, z);
        const double dist = fabs(sqrt(ph + b.R * b.R) - b.R);
        if (dist <= 1.5) {
            const bool inP = ph < 0.0;
#pragma unroll
            for (int i = 1; i < kQ; i++) {
                const bool inQ = sphere_phi(b, x + E3X[i], y + E3Y[i], z + E3Z[i]) < 0.0;
                if (inP != inQ) d[i] += (inP ? 1.0 : -1.0) * W3D[i] * 3.0 * b.F;
            }
        }
    }
#pragma unroll
    for (int i = 0; i < kQ; i++) __builtin_nontemporal_store((float)d[i], B + i * b.plane + row + x);
}

// IB-LBM force field g(x) = sum_k F n_k delta_h(x - X_k) dA, one thread per
// (marker, stencil node), summed in fixed point (the field is built once).
__device__ __forceinline__ double peskin1(double r)
{
    const double a = fabs(r);
    if (a <= 1.0) return (3.0 - 2.0 * a + sqrt(1.0 + 4.0 * a - 4.0 * a * a)) * 0.125;
    if (a <= 2.0) return (5.0 - 2.0 * a - sqrt(-7.0 + 12.0 * a - 4.0 * a * a)) * 0.125;
    return 0.0;
}

__global__ void k_spread3(Box b, const double* __restrict__ X, int N, double dA,
                          long long* __restrict__ g)
{
    const long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (t >= (long long)N * 64) return;
    const int k = (int)(t >> 6), s = (int)(t & 63);
    const double X0 = X[3 * k], Y0 = X[3 * k + 1], Z0 = X[3 * k + 2];
    const int x = (int)floor(X0) - 1 + (s & 3), y = (int)floor(Y0) - 1 + ((s >> 2) & 3),
              z = (int)floor(Z0) - 1 + (s >> 4);
    const double w = peskin1(x - X0) * peskin1(y - Y0) * peskin1(z - Z0);
    if (w == 0.0) return;
    const double nx_ = (X0 - b.cx) / b.R, ny_ = (Y0 - b.cy) / b.R, nz_ = (Z0 - b.cz) / b.R;
    const long long n = (long long)b.nx * b.ny * b.nz;
    const long long c = ((long long)wrapi(z, b.nz) * b.ny + wrapi(y, b.ny)) * b.nx + wrapi(x, b.nx);
    fix3_add(&g[c], b.F * nx_ * w * dA);
    fix3_add(&g[n + c], b.F * ny_ * w * dA);
    fix3_add(&g[2 * n + c], b.F * nz_ * w * dA);
}

// rho, u of f^n (the pulled populations) into out[4][nz][ny][nx] (device).
__global__ void k_fields3(Box b, const float* __restrict__ A, double* __restrict__ out)
{
    const long long n = (long long)b.nx * b.ny * b.nz;
    for (long long c = blockIdx.x * (long long)blockDim.x + threadIdx.x; c < n;
         c += (long long)gridDim.x * blockDim.x) {
        const int x = (int)(c % b.nx), y = (int)((c / b.nx) % b.ny), z = (int)(c / ((long long)b.nx * b.ny));
        double r = 1.0, ux = 0.0, uy = 0.0, uz = 0.0;
        for (int i = 0; i < kQ; i++) {
            const int xs = wrapi(x - E3X[i], b.nx), ys = wrapi(y - E3Y[i], b.ny), zs = wrapi(z - E3Z[i], b.nz);
            const double v = (double)A[i * b.plane + ((long long)zs * b.ny + ys) * b.pitch + xs];
            r += v;
            ux += E3X[i] * v;
            uy += E3Y[i] * v;
            uz += E3Z[i] * v;
        }
        out[c] = r;
        out[n + c] = ux;
        out[2 * n + c] = uy;
        out[3 * n + c] = uz;
    }
}

// stored_i(x) = f_i(x + e_i) - w_i, so that the next pull yields f.
__global__ void k_set3(Box b, const double* __restrict__ f, float* __restrict__ A)
{
    const long long n = (long long)b.nx * b.ny * b.nz;
    for (long long c = blockIdx.x * (long long)blockDim.x + threadIdx.x; c < n;
         c += (long long)gridDim.x * blockDim.x) {
        const int x = (int)(c % b.nx), y = (int)((c / b.nx) % b.ny), z = (int)(c / ((long long)b.nx * b.ny));
        for (int i = 0; i < kQ; i++) {
            const int xd = wrapi(x + E3X[i], b.nx), yd = wrapi(y + E3Y[i], b.ny), zd = wrapi(z + E3Z[i], b.nz);
            const double v = f[i * n + ((long long)zd * b.ny + yd) * b.nx + xd] - W3D[i];
            A[i * b.plane + ((long long)z * b.ny + y) * b.pitch + x] = (float)v;
        }
    }
}

__global__ void k_zero3(float* p, long long n)
{
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x)
        p[i] = 0.f;
}

// ---------------------------------------------------------------------------
// A fixed closed triangulated surface.  Vertices snapped to 2^-16 lu arrive as
// int64; side tests are exact integer determinants.  The host's validation
// (edges at most 4 lu, vertices in [2, n - 3]) keeps every coordinate
// difference below 2^19 and so every determinant below 2^58.  Ties are broken
// by translating the lattice by (e, e^2, e^3), e -> 0+: a node in a face's
// plane takes the side of the plane normal's first non-zero component, a link
// through an edge the side of the first non-zero component of
// (link x edge), so each perturbed crossing of a closed surface is seen by
// exactly one triangle.
struct MeshRec3 {
    int16_t x, y, z;        // sending node
    int8_t dir, sigma;      // population, +1 when the sending node is inside
    int32_t tri;
    float delta;            // sigma w_i [[p]] / c_s^2, added to the stored population
    double jp;              // [[p]] at the crossing
};
static_assert(sizeof(MeshRec3) == 24, "record layout");

constexpr int kMeshWaves = 4;   // triangles per 256-thread block

__device__ __forceinline__ int sgn64(long long v) { return (v > 0) - (v < 0); }

// One wave per triangle: every link P -> P + e_i with P in the triangle's
// node box widened by one.  The wave first finds the plane side of every node
// of the box widened by two (one determinant N . (P - A) per node, N the
// triangle's normal) and keeps it in LDS; a link then needs the edge tests
// only when its two ends lie on different sides.
constexpr int kSideBox = 10;      // nodes per axis: bbox side <= 4 lu -> <= 8 senders + 2
constexpr int kBlockRecs = 256;   // records staged in LDS per block before one global reservation

__global__ __launch_bounds__(256) void k_mesh_links3(const long long* __restrict__ S,
                                                     const int* __restrict__ tri,
                                                     const double* __restrict__ pv, int nt,
                                                     MeshRec3* __restrict__ out, int cap,
                                                     int* __restrict__ count, const int* err)
{
    __shared__ int8_t side[kMeshWaves][kSideBox * kSideBox * kSideBox];
    __shared__ MeshRec3 stage[kBlockRecs];
    __shared__ int n_stage, g_base;
    const int wv = threadIdx.x / 64;
    const int t = blockIdx.x * kMeshWaves + wv;
    const int lane = threadIdx.x % 64;
    if (threadIdx.x == 0) n_stage = 0;
    bool active = t < nt && !(err && *(volatile const int*)err);
    int ia = 0, ib = 0, ic = 0;
    long long A[3] = {0, 0, 0}, B[3] = {0, 0, 0}, C[3] = {0, 0, 0};
    int lo[3] = {0, 0, 0}, n[3] = {0, 0, 0};
    if (active) {
        ia = tri[3 * t]; ib = tri[3 * t + 1]; ic = tri[3 * t + 2];
        for (int k = 0; k < 3; k++) {
            A[k] = S[3 * ia + k]; B[k] = S[3 * ib + k]; C[k] = S[3 * ic + k];
            const long long mn = min(A[k], min(B[k], C[k])), mx = max(A[k], max(B[k], C[k]));
            lo[k] = (int)(mn >> 16) - 1;
            n[k] = (int)((mx + 65535) >> 16) + 1 - lo[k] + 1;
            if (n[k] > kSideBox - 2) active = false;     // span over 4 lu: the caller's bound broken
        }
        if (!active && err) atomicOr((int*)err, 1);
    }
    if (active) {
        // sides of the nodes lo - 1 .. lo + n (every end of every link)
        const long long ux = B[0] - A[0], uy = B[1] - A[1], uz = B[2] - A[2];
        const long long vx = C[0] - A[0], vy = C[1] - A[1], vz = C[2] - A[2];
        const long long Nx = uy * vz - uz * vy, Ny = uz * vx - ux * vz, Nz = ux * vy - uy * vx;
        const int tie = Nx ? sgn64(Nx) : (Ny ? sgn64(Ny) : sgn64(Nz));
        const int m0 = n[0] + 2, m1 = n[1] + 2, m2 = n[2] + 2;
        for (int k = lane; k < m0 * m1 * m2; k += 64) {
            const int ex = k % m0, ey = (k / m0) % m1, ez = k / (m0 * m1);
            const long long px = ((long long)(lo[0] - 1 + ex) << 16) - A[0];
            const long long py = ((long long)(lo[1] - 1 + ey) << 16) - A[1];
            const long long pz = ((long long)(lo[2] - 1 + ez) << 16) - A[2];
            const int sd = sgn64(Nx * px + Ny * py + Nz * pz);
            side[wv][(ez * kSideBox + ey) * kSideBox + ex] = (int8_t)(sd ? sd : tie);
        }
    }
    __syncthreads();
    if (active) {
        // Edge tests.  With P = 2^16 p and E = B - A, the determinant
        // det[2^16 d, A - P, B - P] is 2^16 d . (A x B - 2^16 (p x E)): A x B
        // once per triangle, p x E once per node, then only sums of components
        // for the directions d (entries 0, +-1).  The weights below lack the
        // common factor 2^16, which scales [[p]]'s numerator and denominator
        // alike (exactly).
        const long long* V[3] = {A, B, C};
        long long AB[3][3], E[3][3];
#pragma unroll
        for (int q = 0; q < 3; q++) {
            const long long* a = V[q];
            const long long* b = V[(q + 1) % 3];
            AB[q][0] = a[1] * b[2] - a[2] * b[1];
            AB[q][1] = a[2] * b[0] - a[0] * b[2];
            AB[q][2] = a[0] * b[1] - a[1] * b[0];
            for (int k = 0; k < 3; k++) E[q][k] = b[k] - a[k];
        }
        const int nn = n[0] * n[1] * n[2];
        for (int node = lane; node < nn; node += 64) {
            const int ox = node % n[0], oy = (node / n[0]) % n[1], oz = node / (n[0] * n[1]);
            const int x = lo[0] + ox, y = lo[1] + oy, z = lo[2] + oz;
            const int sp = side[wv][((oz + 1) * kSideBox + oy + 1) * kSideBox + ox + 1];
            long long cr[3][3];        // (A - P) x (B - P) per edge, exact
#pragma unroll
            for (int q = 0; q < 3; q++) {
                const long long pe0 = (long long)y * E[q][2] - (long long)z * E[q][1];
                const long long pe1 = (long long)z * E[q][0] - (long long)x * E[q][2];
                const long long pe2 = (long long)x * E[q][1] - (long long)y * E[q][0];
                cr[q][0] = AB[q][0] - (pe0 << 16);
                cr[q][1] = AB[q][1] - (pe1 << 16);
                cr[q][2] = AB[q][2] - (pe2 << 16);
            }
#pragma unroll 1
            for (int i = 1; i < kQ; i++) {
                const int dx = E3X[i], dy = E3Y[i], dz = E3Z[i];
                const int sq = side[wv][((oz + 1 + dz) * kSideBox + oy + 1 + dy) * kSideBox + ox + 1 + dx];
                if (sp == sq) continue;
                long long wq[3];
                int es[3];
#pragma unroll
                for (int q = 0; q < 3; q++) {
                    wq[q] = dx * cr[q][0] + dy * cr[q][1] + dz * cr[q][2];
                    if (wq[q]) {
                        es[q] = sgn64(wq[q]);
                    } else {      // tie: the sign of d x E, first non-zero component
                        const long long c0 = dy * E[q][2] - dz * E[q][1];
                        const long long c1 = dz * E[q][0] - dx * E[q][2];
                        const long long c2 = dx * E[q][1] - dy * E[q][0];
                        es[q] = c0 ? sgn64(c0) : (c1 ? sgn64(c1) : sgn64(c2));
                    }
                }
                if (es[0] != es[1] || es[1] != es[2]) continue;
                // edge (A, B) weighs C, (B, C) weighs A, (C, A) weighs B
                const double lc = (double)wq[0], la = (double)wq[1], lb = (double)wq[2];
                const double jp = (la * pv[ia] + lb * pv[ib] + lc * pv[ic]) / (la + lb + lc);
                const int sigma = sp < 0 ? 1 : -1;
                MeshRec3 r;
                r.x = (int16_t)x; r.y = (int16_t)y; r.z = (int16_t)z;
                r.dir = (int8_t)i; r.sigma = (int8_t)sigma; r.tri = t;
                r.delta = (float)(sigma * W3D[i] * jp * 3.0);
                r.jp = jp;
                const int sl = atomicAdd(&n_stage, 1);
                if (sl < kBlockRecs) {
                    stage[sl] = r;
                } else {                 // a crowded block: straight to global memory
                    const int slot = atomicAdd(count, 1);
                    if (slot < cap) out[slot] = r;
                }
            }
        }
    }
    __syncthreads();
    const int staged = min(n_stage, kBlockRecs);
    if (threadIdx.x == 0) g_base = staged ? atomicAdd(count, staged) : 0;
    __syncthreads();
    for (int k = threadIdx.x; k < staged; k += blockDim.x)
        if (g_base + k < cap) out[g_base + k] = stage[k];
}

// After the sweep: the stored population of every cut link's sending node
// takes the link's jump, so the next pull carries it across.  The targets are
// distinct (links that cross twice were merged on the host) and in address
// order, so a plain read-modify-write suffices and neighbouring lanes share
// cache lines.
__global__ void k_mesh_apply3(const long long* __restrict__ off, const float* __restrict__ delta, int n,
                              float* __restrict__ B)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    const long long o = off[k];
    B[o] += delta[k];
}

// ---------------------------------------------------------------------------
// A deformable triangulated membrane under surface tension.  Every kernel
// reads the sticky error word first and does nothing once it is set, so a
// surface that leaves the supported region stops the membrane work of every
// later step (the fluid sweep still runs).  err: 1 geometry, 2 capacity.
__device__ __forceinline__ bool memb_failed(const int* err) { return *(volatile const int*)err != 0; }

__device__ __forceinline__ bool memb_inside(const Box& b, double x, double y, double z)
{
    return x >= 2.0 && x <= b.nx - 3.0 && y >= 2.0 && y <= b.ny - 3.0 && z >= 2.0 && z <= b.nz - 3.0;
}

// A free rigid sphere: state c, U, a, W, wdot, Uprev, Wprev; the last step's
// force and torque; dc, the centre's step (the vertices follow it).
struct Body3 {
    double c[3], U[3], a[3], W[3], wd[3], Up[3], Wp[3];
    double F[3], T[3], dc[3];
};

// U_v = sum of u(x) delta_h(x - X_v) over the 4 x 4 x 4 nodes around X_v: one
// wave per vertex, one lane per node, u from the pulled deviations.
__global__ __launch_bounds__(256) void k_memb_interp3(Box b, const float* __restrict__ A,
                                                      const double* __restrict__ X, int nv,
                                                      double* __restrict__ U, int* err)
{
    const int v = blockIdx.x * 4 + threadIdx.x / 64;
    const int lane = threadIdx.x % 64;
    if (v >= nv || memb_failed(err)) return;
    const double X0 = X[3 * v], Y0 = X[3 * v + 1], Z0 = X[3 * v + 2];
    if (!memb_inside(b, X0, Y0, Z0)) {
        if (lane == 0) atomicOr(err, 1);
        return;
    }
    const int x0 = (int)floor(X0) - 1, y0 = (int)floor(Y0) - 1, z0 = (int)floor(Z0) - 1;
    const int x = x0 + (lane & 3), y = y0 + ((lane >> 2) & 3), z = z0 + (lane >> 4);
    const double w = peskin1(x - X0) * peskin1(y - Y0) * peskin1(z - Z0);
    double jx = 0.0, jy = 0.0, jz = 0.0;
#pragma unroll
    for (int i = 0; i < kQ; i++) {
        const int xs = wrapi(x - E3X[i], b.nx), ys = wrapi(y - E3Y[i], b.ny), zs = wrapi(z - E3Z[i], b.nz);
        const double d = (double)A[i * b.plane + ((long long)zs * b.ny + ys) * b.pitch + xs];
        jx += E3X[i] * d;
        jy += E3Y[i] * d;
        jz += E3Z[i] * d;
    }
    double ux = jx * w, uy = jy * w, uz = jz * w;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        ux += __shfl_xor(ux, o, 64);
        uy += __shfl_xor(uy, o, 64);
        uz += __shfl_xor(uz, o, 64);
    }
    if (lane == 0) {
        U[3 * v] = ux;
        U[3 * v + 1] = uy;
        U[3 * v + 2] = uz;
    }
}

// Vertices snapped to 2^-16 for the exact link tests, after the bounds check.
__global__ void k_memb_snap3(Box b, const double* __restrict__ X, int nv, long long* __restrict__ S, int* err)
{
    const int v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= nv || memb_failed(err)) return;
    const double x = X[3 * v], y = X[3 * v + 1], z = X[3 * v + 2];
    if (!memb_inside(b, x, y, z)) {
        atomicOr(err, 1);
        return;
    }
    S[3 * v] = __double2ll_rn(x * 65536.0);
    S[3 * v + 1] = __double2ll_rn(y * 65536.0);
    S[3 * v + 2] = __double2ll_rn(z * 65536.0);
}

// Per vertex, over its triangles in ascending order: the tension force on the
// fluid G_v = -gamma sum dA_t/dX_v with dA/da = (1/2) nhat x (c - b) for a
// triangle (a, b, c), cyclically; the area-weighted normal; the vertex area
// (a third of each triangle); then [[p]]_v = G.n / A_v and the tangential
// part.  Edges longer than 4 lu or a degenerate triangle set the error.
// law 1 (a fixed rigid surface, direct forcing to rest): G_v = (0 - U_v) A_v
// instead of the tension force.  G (the force on the fluid) is kept for the
// force on the surface.
__global__ void k_memb_forces3(const double* __restrict__ X, const int* __restrict__ tri,
                               const int* __restrict__ vt_off, const int* __restrict__ vt, int nv,
                               double gamma, int law, const double* __restrict__ U, double* __restrict__ jp,
                               double* __restrict__ Gt, double* __restrict__ Gout, const Body3* __restrict__ body,
                               int* err)
{
    const int v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= nv || memb_failed(err)) return;
    double G[3] = {0.0, 0.0, 0.0}, nr[3] = {0.0, 0.0, 0.0}, Av = 0.0;
    for (int q = vt_off[v]; q < vt_off[v + 1]; q++) {
        const int t = vt[q];
        const int c3[3] = {tri[3 * t], tri[3 * t + 1], tri[3 * t + 2]};
        const int j = c3[0] == v ? 0 : (c3[1] == v ? 1 : 2);
        const double* a = X + 3 * c3[0];
        const double* bb = X + 3 * c3[1];
        const double* c = X + 3 * c3[2];
        double u[3], w[3];
        for (int k = 0; k < 3; k++) {
            u[k] = bb[k] - a[k];
            w[k] = c[k] - a[k];
        }
        const double l2c = (c[0] - bb[0]) * (c[0] - bb[0]) + (c[1] - bb[1]) * (c[1] - bb[1]) +
                           (c[2] - bb[2]) * (c[2] - bb[2]);
        // 15.9 lu^2 keeps the snapped span of every triangle within 4 lu per axis
        if (u[0] * u[0] + u[1] * u[1] + u[2] * u[2] > 15.9 || w[0] * w[0] + w[1] * w[1] + w[2] * w[2] > 15.9 ||
            l2c > 15.9) {
            atomicOr(err, 1);
            return;
        }
        const double N[3] = {u[1] * w[2] - u[2] * w[1], u[2] * w[0] - u[0] * w[2], u[0] * w[1] - u[1] * w[0]};
        const double len = sqrt(N[0] * N[0] + N[1] * N[1] + N[2] * N[2]);
        if (!(len > 0.0)) {
            atomicOr(err, 1);
            return;
        }
        const double nh[3] = {N[0] / len, N[1] / len, N[2] / len};
        const double* p = X + 3 * c3[(j + 1) % 3];
        const double* qq = X + 3 * c3[(j + 2) % 3];
        const double e[3] = {qq[0] - p[0], qq[1] - p[1], qq[2] - p[2]};
        const double dA[3] = {0.5 * (nh[1] * e[2] - nh[2] * e[1]), 0.5 * (nh[2] * e[0] - nh[0] * e[2]),
                              0.5 * (nh[0] * e[1] - nh[1] * e[0])};
        for (int k = 0; k < 3; k++) {
            G[k] -= gamma * dA[k];
            nr[k] += N[k];
        }
        Av += len / 6.0;
    }
    const double l = sqrt(nr[0] * nr[0] + nr[1] * nr[1] + nr[2] * nr[2]);
    for (int k = 0; k < 3; k++) nr[k] /= l;
    if (law == 1)
        for (int k = 0; k < 3; k++) G[k] = (0.0 - U[3 * v + k]) * Av;
    if (law == 3) {   // free rigid sphere: U^D = U_b + W x (X_v - c)
        const double rx = X[3 * v] - body->c[0], ry = X[3 * v + 1] - body->c[1], rz = X[3 * v + 2] - body->c[2];
        const double ud[3] = {body->U[0] + body->W[1] * rz - body->W[2] * ry,
                              body->U[1] + body->W[2] * rx - body->W[0] * rz,
                              body->U[2] + body->W[0] * ry - body->W[1] * rx};
        for (int k = 0; k < 3; k++) G[k] = (ud[k] - U[3 * v + k]) * Av;
    }
    const double gn = G[0] * nr[0] + G[1] * nr[1] + G[2] * nr[2];
    // law 2 (IB-LBM membrane): the whole force is spread and there is no jump
    jp[v] = law == 2 ? 0.0 : gn / Av;
    for (int k = 0; k < 3; k++) {
        Gt[3 * v + k] = law == 2 ? G[k] : G[k] - gn * nr[k];
        Gout[3 * v + k] = G[k];
    }
}

// g(x) += Gt_v delta_h(x - X_v): one thread per (vertex, stencil node).
__global__ void k_memb_spread3(Box b, const double* __restrict__ X, const double* __restrict__ Gt, int nv,
                               long long* __restrict__ g, const int* err)
{
    const long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (t >= (long long)nv * 64 || memb_failed(err)) return;
    const int v = (int)(t / 64), lane = (int)(t % 64);
    const double X0 = X[3 * v], Y0 = X[3 * v + 1], Z0 = X[3 * v + 2];
    const int x = (int)floor(X0) - 1 + (lane & 3), y = (int)floor(Y0) - 1 + ((lane >> 2) & 3),
              z = (int)floor(Z0) - 1 + (lane >> 4);
    const double w = peskin1(x - X0) * peskin1(y - Y0) * peskin1(z - Z0);
    const long long n = (long long)b.nx * b.ny * b.nz;
    const long long c = ((long long)z * b.ny + y) * b.nx + x;
    fix3_add(&g[c], Gt[3 * v] * w);
    fix3_add(&g[n + c], Gt[3 * v + 1] * w);
    fix3_add(&g[2 * n + c], Gt[3 * v + 2] * w);
}

// IB-LBM membrane (law 2): the vertices move with the velocity of the
// distributions after the step's force, so the spread force g (and the
// uniform body force) interpolated at each vertex joins U_v; one wave per
// vertex, one lane per stencil node.
__global__ __launch_bounds__(256) void k_memb_addg3(Box b, const double* __restrict__ X, int nv,
                                                    const long long* __restrict__ g, double bx, double by,
                                                    double bz, double* __restrict__ U, const int* err)
{
    const int v = blockIdx.x * 4 + threadIdx.x / 64;
    const int lane = threadIdx.x % 64;
    if (v >= nv || memb_failed(err)) return;
    const double X0 = X[3 * v], Y0 = X[3 * v + 1], Z0 = X[3 * v + 2];
    const int x = (int)floor(X0) - 1 + (lane & 3), y = (int)floor(Y0) - 1 + ((lane >> 2) & 3),
              z = (int)floor(Z0) - 1 + (lane >> 4);
    const double w = peskin1(x - X0) * peskin1(y - Y0) * peskin1(z - Z0);
    const long long n = (long long)b.nx * b.ny * b.nz;
    const long long c = ((long long)z * b.ny + y) * b.nx + x;
    double gx = fix3_get(g[c]) * w, gy = fix3_get(g[n + c]) * w, gz = fix3_get(g[2 * n + c]) * w;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        gx += __shfl_xor(gx, o, 64);
        gy += __shfl_xor(gy, o, 64);
        gz += __shfl_xor(gz, o, 64);
    }
    if (lane == 0) {
        U[3 * v] += gx + bx;
        U[3 * v + 1] += gy + by;
        U[3 * v + 2] += gz + bz;
    }
}

// One block: F = -sum G_v + V_s (U - Uprev), T = -sum r_v x G_v +
// (I_s / rho*) (W - Wprev) over the vertices (a fixed reduction order), then
// the update of Sec. 2.3: a = F / m, U += a, c += U + (a_old + a) / 2,
// W += T / I_s.
__global__ __launch_bounds__(1024) void k_body3(const double* __restrict__ X, const double* __restrict__ G, int nv,
                                                double radius, double rho_star, Body3* __restrict__ b, const int* err)
{
    __shared__ double red[6][1024];
    if (memb_failed(err)) return;
    const double cx = b->c[0], cy = b->c[1], cz = b->c[2];
    double acc[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    for (int v = threadIdx.x; v < nv; v += blockDim.x) {
        const double rx = X[3 * v] - cx, ry = X[3 * v + 1] - cy, rz = X[3 * v + 2] - cz;
        const double gx = G[3 * v], gy = G[3 * v + 1], gz = G[3 * v + 2];
        acc[0] -= gx;
        acc[1] -= gy;
        acc[2] -= gz;
        acc[3] -= ry * gz - rz * gy;
        acc[4] -= rz * gx - rx * gz;
        acc[5] -= rx * gy - ry * gx;
    }
    for (int k = 0; k < 6; k++) red[k][threadIdx.x] = acc[k];
    __syncthreads();
    for (int o = blockDim.x / 2; o > 0; o >>= 1) {
        if (threadIdx.x < o)
            for (int k = 0; k < 6; k++) red[k][threadIdx.x] += red[k][threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x != 0) return;
    const double Vs = 4.0 * M_PI * radius * radius * radius / 3.0, m = rho_star * Vs;
    const double Is = 0.4 * m * radius * radius;
    for (int k = 0; k < 3; k++) {
        const double F = red[k][0] + Vs * (b->U[k] - b->Up[k]);
        const double T = red[3 + k][0] + Is / rho_star * (b->W[k] - b->Wp[k]);
        const double an = F / m, wn = T / Is;
        b->F[k] = F;
        b->T[k] = T;
        b->Up[k] = b->U[k];
        b->Wp[k] = b->W[k];
        const double dc = b->U[k] + 0.5 * (b->a[k] + an);
        b->dc[k] = dc;
        b->c[k] += dc;
        b->U[k] += an;
        b->a[k] = an;
        b->W[k] += wn;
        b->wd[k] = wn;
    }
}

__global__ void k_body_move3(double* __restrict__ X, int nv, const Body3* __restrict__ b, const int* err)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= 3 * nv || memb_failed(err)) return;
    X[k] += b->dc[k % 3];
}

// After the sweep has read the force field: zero the stencils the spread of
// this step wrote (the same vertices, before they move), so the field starts
// the next step at zero without clearing the whole box.  It ignores the
// error word (a stop after the spread must not leave its forces behind) and
// skips vertices outside the region, which were never spread.
__global__ void k_memb_unspread3(Box b, const double* __restrict__ X, int nv, long long* __restrict__ g)
{
    const long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (t >= (long long)nv * 64) return;
    const int v = (int)(t / 64), lane = (int)(t % 64);
    const double X0 = X[3 * v], Y0 = X[3 * v + 1], Z0 = X[3 * v + 2];
    if (!memb_inside(b, X0, Y0, Z0)) return;
    const int x = (int)floor(X0) - 1 + (lane & 3), y = (int)floor(Y0) - 1 + ((lane >> 2) & 3),
              z = (int)floor(Z0) - 1 + (lane >> 4);
    const long long n = (long long)b.nx * b.ny * b.nz;
    const long long c = ((long long)z * b.ny + y) * b.nx + x;
    g[c] = 0;
    g[n + c] = 0;
    g[2 * n + c] = 0;
}

__global__ void k_zero_count3(int* count) { *count = 0; }

// The step's jumps, added to the stored populations independently of the
// records' order: the deltas of the records (several may share a target
// population) are summed per target in fixed point (fix3) in an open-
// addressing table, then each distinct target takes its sum in one
// read-modify-write, which also empties its table entry for the next step.
constexpr unsigned long long kEmpty3 = ~0ull;
constexpr int kProbe3 = 256;

__device__ __forceinline__ unsigned hash3(unsigned long long key, int bits)
{
    return (unsigned)((key * 0x9E3779B97F4A7C15ull) >> (64 - bits));
}

__global__ void k_memb_accum3(Box b, const MeshRec3* __restrict__ r, const int* __restrict__ count, int cap,
                              unsigned long long* __restrict__ keys, long long* __restrict__ sums, int bits,
                              int* __restrict__ used, int* __restrict__ n_used, int* err)
{
    if (memb_failed(err)) return;
    const int n = *count;
    if (n > cap) {
        if (blockIdx.x == 0 && threadIdx.x == 0) atomicOr(err, 2);
        return;
    }
    const unsigned mask = (1u << bits) - 1u;
    for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < n; k += gridDim.x * blockDim.x) {
        const MeshRec3 q = r[k];
        const unsigned long long key =
            (unsigned long long)(q.dir * b.plane + ((long long)q.z * b.ny + q.y) * b.pitch + q.x);
        // the table has twice as many entries as there can be records; a
        // probe that finds neither the key nor a free entry within kProbe3
        // steps (no realistic load comes near) reports a capacity error
        unsigned sl = hash3(key, bits);
        bool found = false;
        for (int t = 0; t < kProbe3; t++) {
            const unsigned long long prev = atomicCAS(&keys[sl], kEmpty3, key);
            if (prev == kEmpty3) {
                const int u = atomicAdd(n_used, 1);
                if (u < cap) used[u] = (int)sl;
                found = u < cap;
                break;
            }
            if (prev == key) {
                found = true;
                break;
            }
            sl = (sl + 1u) & mask;
        }
        if (!found) {
            atomicOr(err, 2);
            continue;
        }
        fix3_add(&sums[sl], (double)q.delta);
    }
}

__global__ void k_memb_addsums3(const int* __restrict__ n_used, int cap, const int* __restrict__ used,
                                unsigned long long* __restrict__ keys, long long* __restrict__ sums,
                                float* __restrict__ B)
{
    const int n = min(*n_used, cap);
    for (int u = blockIdx.x * blockDim.x + threadIdx.x; u < n; u += gridDim.x * blockDim.x) {
        const int sl = used[u];
        const long long off = (long long)keys[sl];
        B[off] = (float)((double)B[off] + fix3_get(sums[sl]));
        keys[sl] = kEmpty3;
        sums[sl] = 0;
    }
}

__global__ void k_memb_move3(double* __restrict__ X, const double* __restrict__ U, int n3, const int* err)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n3 || memb_failed(err)) return;
    X[k] += U[k];
}

}  // namespace iilbm3

using namespace iilbm3;

struct ii_lbm3_handle {
    ii_lbm3_allocator alloc{};   // device memory from the caller (alloc == NULL: hipMalloc)
    Box b;
    ii_lbm3_problem prob;
    bool mrt = false;
    hipStream_t stream;
    long long* mesh_S = nullptr;      // snapped vertices, int64 [3 n_vert]
    int* mesh_tri = nullptr;
    double* mesh_pv = nullptr;
    MeshRec3* mesh_rec = nullptr;
    int* mesh_count = nullptr;
    int mesh_links = 0;
    long long* apply_off = nullptr;   // distinct target offsets in the lattice, ascending
    float* apply_delta = nullptr;     // summed jumps per target
    int apply_n = 0;
    // deformable membrane (the surface above is then unused)
    bool memb = false;
    int memb_nv = 0, memb_nt = 0, memb_cap = 0;
    double memb_gamma = 0.0;
    double* memb_X = nullptr;         // vertices [3 nv]
    double* memb_U = nullptr;         // velocities of the last step [3 nv]
    double* memb_jp = nullptr;        // [[p]] per vertex
    double* memb_Gt = nullptr;        // tangential force per vertex [3 nv]
    double* memb_G = nullptr;         // force on the fluid per vertex [3 nv]
    int memb_law = 0;                 // 0 tension membrane, 1 fixed rigid surface, 2 IB membrane, 3 free sphere
    Body3* body3 = nullptr;           // law 3: the sphere's state
    double body3_radius = 0.0, body3_rho = 0.0;
    long long* memb_S = nullptr;      // snapped vertices
    int* memb_tri = nullptr;
    int* memb_vt_off = nullptr;       // triangles of each vertex (CSR, ascending)
    int* memb_vt = nullptr;
    MeshRec3* memb_rec = nullptr;
    int* memb_count = nullptr;
    // per-target sums of the jumps (k_memb_accum3): 2^memb_hbits entries
    unsigned long long* memb_hkeys = nullptr;
    long long* memb_hsums = nullptr;
    int* memb_used = nullptr;       // table entries in use (memb_cap)
    int* memb_nused = nullptr;
    int memb_hbits = 0;
    int* memb_err = nullptr;
    float* lat[2] = {nullptr, nullptr};
    long long* g = nullptr;    // spread force field, fixed point (fix3)
    int parity = 0;
    bool timing = false;
    std::vector<hipEvent_t> ev;
    int ev_used = 0;
    double ms = 0.0;
    long long launches = 0;
};

static int fail3(hipError_t e) { return e == hipSuccess ? II_LBM_OK : II_LBM_EDEVICE; }

// Every device buffer of a handle comes from here: the caller's allocator
// when it gave one (ii_lbm3_init_with), hipMalloc otherwise.  Buffers are
// returned only after the handle's stream has finished with them.
template <class T>
static hipError_t dmalloc(ii_lbm3_handle* h, T** p, size_t bytes)
{
    if (!h->alloc.alloc) return hipMalloc((void**)p, bytes);
    *p = (T*)h->alloc.alloc(bytes, h->alloc.ctx);
    return *p ? hipSuccess : hipErrorOutOfMemory;
}

static void dfree(ii_lbm3_handle* h, void* p)
{
    if (!p) return;
    if (h->alloc.release)
        h->alloc.release(p, h->alloc.ctx);
    else
        (void)hipFree(p);
}

static void free_mesh(ii_lbm3_handle* h)
{
    for (void* q : {(void*)h->mesh_S, (void*)h->mesh_tri, (void*)h->mesh_pv, (void*)h->mesh_rec,
                    (void*)h->mesh_count, (void*)h->apply_off, (void*)h->apply_delta})
        dfree(h, q);
    h->mesh_S = nullptr; h->mesh_tri = nullptr; h->mesh_pv = nullptr; h->mesh_rec = nullptr;
    h->mesh_count = nullptr; h->mesh_links = 0;
    h->apply_off = nullptr; h->apply_delta = nullptr; h->apply_n = 0;
}

static long long snap_2m16(double v) { return llrint(v * 65536.0); }

static void free_membrane(ii_lbm3_handle* h)
{
    for (void* q : {(void*)h->memb_X, (void*)h->memb_U, (void*)h->memb_jp, (void*)h->memb_Gt, (void*)h->memb_G,
                    (void*)h->memb_S,
                    (void*)h->memb_tri, (void*)h->memb_vt_off, (void*)h->memb_vt, (void*)h->memb_rec,
                    (void*)h->memb_count, (void*)h->memb_err, (void*)h->memb_hkeys, (void*)h->memb_hsums,
                    (void*)h->memb_used, (void*)h->memb_nused})
        dfree(h, q);
    h->memb_hkeys = nullptr;
    h->memb_hsums = nullptr;
    h->memb_used = h->memb_nused = nullptr;
    h->memb_hbits = 0;
    h->memb_X = h->memb_U = h->memb_jp = h->memb_Gt = h->memb_G = nullptr;
    h->memb_law = 0;
    dfree(h, h->body3);
    h->body3 = nullptr;
    h->memb_S = nullptr;
    h->memb_tri = h->memb_vt_off = h->memb_vt = h->memb_count = h->memb_err = nullptr;
    h->memb_rec = nullptr;
    h->memb = false;
    h->memb_nv = h->memb_nt = h->memb_cap = 0;
}

// One membrane step's work before the sweep (interpolation, forces, spread,
// links) and after it (jumps, motion).
static void memb_before_sweep(ii_lbm3_handle* h, const float* A)
{
    const Box& b = h->b;
    const int nv = h->memb_nv, nt = h->memb_nt;
    hipLaunchKernelGGL(k_memb_interp3, dim3((nv + 3) / 4), dim3(256), 0, h->stream, b, A, h->memb_X, nv,
                       h->memb_U, h->memb_err);
    hipLaunchKernelGGL(k_memb_snap3, dim3((nv + 255) / 256), dim3(256), 0, h->stream, b, h->memb_X, nv,
                       h->memb_S, h->memb_err);
    hipLaunchKernelGGL(k_memb_forces3, dim3((nv + 255) / 256), dim3(256), 0, h->stream, h->memb_X, h->memb_tri,
                       h->memb_vt_off, h->memb_vt, nv, (h->memb_law == 1 || h->memb_law == 3) ? 0.0 : h->memb_gamma,
                       h->memb_law, (const double*)h->memb_U, h->memb_jp, h->memb_Gt, h->memb_G,
                       (const Body3*)h->body3, h->memb_err);
    hipLaunchKernelGGL(k_memb_spread3, dim3((unsigned)(((long long)nv * 64 + 255) / 256)), dim3(256), 0, h->stream,
                       b, h->memb_X, h->memb_Gt, nv, h->g, h->memb_err);
    if (h->memb_law == 2) {                                       // IB-LBM: no jumps
        hipLaunchKernelGGL(k_memb_addg3, dim3((nv + 3) / 4), dim3(256), 0, h->stream, b,
                           (const double*)h->memb_X, nv, (const long long*)h->g, b.g[0], b.g[1],
                           b.g[2], h->memb_U, (const int*)h->memb_err);
        return;
    }
    hipLaunchKernelGGL(k_zero_count3, dim3(1), dim3(1), 0, h->stream, h->memb_count);
    hipLaunchKernelGGL(k_mesh_links3, dim3((nt + kMeshWaves - 1) / kMeshWaves), dim3(256), 0, h->stream,
                       h->memb_S, h->memb_tri, h->memb_jp, nt, h->memb_rec, h->memb_cap, h->memb_count,
                       (const int*)h->memb_err);
}

static void memb_after_sweep(ii_lbm3_handle* h, float* B)
{
    if (h->memb_law != 2) {
        const dim3 grid(std::min((h->memb_cap + 255) / 256, 2048));
        hipLaunchKernelGGL(k_zero_count3, dim3(1), dim3(1), 0, h->stream, h->memb_nused);
        hipLaunchKernelGGL(k_memb_accum3, grid, dim3(256), 0, h->stream, h->b, (const MeshRec3*)h->memb_rec,
                           (const int*)h->memb_count, h->memb_cap, h->memb_hkeys, h->memb_hsums, h->memb_hbits,
                           h->memb_used, h->memb_nused, h->memb_err);
        hipLaunchKernelGGL(k_memb_addsums3, grid, dim3(256), 0, h->stream, (const int*)h->memb_nused,
                           h->memb_cap, (const int*)h->memb_used, h->memb_hkeys, h->memb_hsums, B);
    }
    hipLaunchKernelGGL(k_memb_unspread3, dim3((unsigned)(((long long)h->memb_nv * 64 + 255) / 256)), dim3(256), 0,
                       h->stream, h->b, (const double*)h->memb_X, h->memb_nv, h->g);
    if (h->memb_law == 0 || h->memb_law == 2)
        hipLaunchKernelGGL(k_memb_move3, dim3((3 * h->memb_nv + 255) / 256), dim3(256), 0, h->stream, h->memb_X,
                           h->memb_U, 3 * h->memb_nv, h->memb_err);
    if (h->memb_law == 3) {
        hipLaunchKernelGGL(k_body3, dim3(1), dim3(1024), 0, h->stream, (const double*)h->memb_X,
                           (const double*)h->memb_G, h->memb_nv, h->body3_radius, h->body3_rho, h->body3,
                           h->memb_err);
        hipLaunchKernelGGL(k_body_move3, dim3((3 * h->memb_nv + 255) / 256), dim3(256), 0, h->stream, h->memb_X,
                           h->memb_nv, (const Body3*)h->body3, h->memb_err);
    }
}

extern "C" {

int ii_lbm3_init(const ii_lbm3_problem* p, const double* X0, void* hip_stream, ii_lbm3_handle** out)
{
    return ii_lbm3_init_with(p, X0, hip_stream, nullptr, out);
}

int ii_lbm3_init_with(const ii_lbm3_problem* p, const double* X0, void* hip_stream,
                      const ii_lbm3_allocator* alloc, ii_lbm3_handle** out)
{
    if (!p || !out) return II_LBM_EINVAL;
    *out = nullptr;
    if (alloc && (!alloc->alloc || !alloc->release)) return II_LBM_EINVAL;
    if (p->nx < 8 || p->ny < 8 || p->nz < 8 || p->nx > 1024 || p->ny > 1024 || p->nz > 1024)
        return II_LBM_EINVAL;
    if (!(p->tau > 0.5) || !isfinite(p->tau)) return II_LBM_EINVAL;
    if (p->force_mode != II_LBM_FORCE_II && p->force_mode != II_LBM_FORCE_IB) return II_LBM_EINVAL;
    if (p->collision != II_LBM_SRT && p->collision != II_LBM_MRT) return II_LBM_EINVAL;
    const bool sphere = p->radius > 0.0;
    if (sphere) {
        const double c[3] = {p->center[0], p->center[1], p->center[2]};
        const int n[3] = {p->nx, p->ny, p->nz};
        for (int a = 0; a < 3; a++)
            if (!(c[a] - p->radius >= 3.0 && c[a] + p->radius <= n[a] - 4.0)) return II_LBM_EGEOMETRY;
        if (!isfinite(p->f_normal)) return II_LBM_EINVAL;
        if (p->force_mode == II_LBM_FORCE_IB) {
            if (p->n_markers < 4 || !X0) return II_LBM_EINVAL;
            // the spread's 4 x 4 x 4 stencil must stay one wrap from the box
            for (int k = 0; k < p->n_markers; k++)
                for (int a = 0; a < 3; a++) {
                    const double v = X0[3 * k + a];
                    if (!isfinite(v)) return II_LBM_EINVAL;
                    if (!(v >= 2.0 && v <= n[a] - 3.0)) return II_LBM_EGEOMETRY;
                }
        }
    }
    ii_lbm3_handle* h = new ii_lbm3_handle();
    if (alloc) h->alloc = *alloc;
    h->prob = *p;
    Box& b = h->b;
    b.nx = p->nx; b.ny = p->ny; b.nz = p->nz;
    b.pitch = (p->nx + 63) / 64 * 64;
    b.plane = (long long)b.pitch * b.ny * b.nz;
    b.omega = 1.0 / p->tau;
    for (int a = 0; a < 3; a++) b.g[a] = p->body_force[a];
    b.sphere = sphere;
    b.ib = sphere && p->force_mode == II_LBM_FORCE_IB;
    b.cx = p->center[0]; b.cy = p->center[1]; b.cz = p->center[2];
    b.R = p->radius; b.F = p->f_normal;
    {
        // rates of the 19 moments: conserved 0; e 1.19; eps, 3pixx, piww 1.4;
        // q 1.2; the viscous stresses 1/tau; m 1.98
        const double sv = 1.0 / p->tau;
        const double rate[kQ] = {0.0, 1.19, 1.4, 0.0, 1.2, 0.0, 1.2, 0.0, 1.2, sv,
                                 1.4, sv,   1.4, sv,  sv,  sv,  1.98, 1.98, 1.98};
        for (int k = 0; k < kQ; k++) {
            double n2 = 0.0;
            for (int i = 0; i < kQ; i++) n2 += (double)kM3.m[k][i] * kM3.m[k][i];
            b.sk[k] = rate[k] / n2;
        }
    }
    h->mrt = p->collision == II_LBM_MRT;
    h->stream = (hipStream_t)hip_stream;
    const size_t lat = (size_t)kQ * b.plane * sizeof(float);
    hipError_t e = dmalloc(h, &h->lat[0], lat);
    if (e == hipSuccess) e = dmalloc(h, &h->lat[1], lat);
    const long long n = (long long)b.nx * b.ny * b.nz;
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_zero3, dim3(2048), dim3(256), 0, h->stream, h->lat[0], (long long)kQ * b.plane);
        hipLaunchKernelGGL(k_zero3, dim3(2048), dim3(256), 0, h->stream, h->lat[1], (long long)kQ * b.plane);
        e = hipGetLastError();
    }
    if (e == hipSuccess && b.ib) {
        e = dmalloc(h, &h->g, (size_t)3 * n * sizeof(long long));
        double* dX = nullptr;
        if (e == hipSuccess) e = hipMemsetAsync(h->g, 0, (size_t)3 * n * sizeof(long long), h->stream);
        if (e == hipSuccess) e = dmalloc(h, &dX, (size_t)3 * p->n_markers * sizeof(double));
        if (e == hipSuccess)
            e = hipMemcpyAsync(dX, X0, (size_t)3 * p->n_markers * sizeof(double), hipMemcpyHostToDevice,
                               h->stream);
        if (e == hipSuccess) {
            const double dA = 4.0 * M_PI * b.R * b.R / p->n_markers;
            const long long threads = (long long)p->n_markers * 64;
            hipLaunchKernelGGL(k_spread3, dim3((unsigned)((threads + 255) / 256)), dim3(256), 0, h->stream, b,
                               dX, p->n_markers, dA, h->g);
            e = hipGetLastError();
        }
        if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
        else (void)hipStreamSynchronize(h->stream);
        dfree(h, dX);
    }
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    if (e != hipSuccess) {
        ii_lbm3_destroy(h);
        return II_LBM_EDEVICE;
    }
    *out = h;
    return II_LBM_OK;
}

int ii_lbm3_step(ii_lbm3_handle* h, int64_t n_steps)
{
    if (!h || n_steps < 0) return II_LBM_EINVAL;
    const Box& b = h->b;
    const dim3 grid((b.nx + kBX - 1) / kBX, b.ny, b.nz);
    for (int64_t s = 0; s < n_steps; s++) {
        const bool t = h->timing;
        if (t) {
            if (h->ev_used + 2 > (int)h->ev.size()) {
                hipEvent_t a, c;
                if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&c) != hipSuccess) return II_LBM_EDEVICE;
                h->ev.push_back(a);
                h->ev.push_back(c);
            }
            (void)hipEventRecord(h->ev[h->ev_used], h->stream);
        }
        float* src = h->lat[h->parity];
        float* dst = h->lat[h->parity ^ 1];
        if (h->memb) {
            memb_before_sweep(h, src);
            if (h->mrt)
                hipLaunchKernelGGL((k_sweep3<true, true>), grid, dim3(kBX), 0, h->stream, b, src, dst, h->g);
            else
                hipLaunchKernelGGL((k_sweep3<true, false>), grid, dim3(kBX), 0, h->stream, b, src, dst, h->g);
        } else if (b.ib && h->mrt)
            hipLaunchKernelGGL((k_sweep3<true, true>), grid, dim3(kBX), 0, h->stream, b, src, dst, h->g);
        else if (b.ib)
            hipLaunchKernelGGL((k_sweep3<true, false>), grid, dim3(kBX), 0, h->stream, b, src, dst, h->g);
        else if (h->mrt)
            hipLaunchKernelGGL((k_sweep3<false, true>), grid, dim3(kBX), 0, h->stream, b, src, dst, h->g);
        else
            hipLaunchKernelGGL((k_sweep3<false, false>), grid, dim3(kBX), 0, h->stream, b, src, dst, h->g);
        if (t) {
            (void)hipEventRecord(h->ev[h->ev_used + 1], h->stream);
            h->ev_used += 2;
        }
        if (h->memb) memb_after_sweep(h, dst);
        if (h->apply_n > 0)
            hipLaunchKernelGGL(k_mesh_apply3, dim3((h->apply_n + 255) / 256), dim3(256), 0, h->stream,
                               h->apply_off, h->apply_delta, h->apply_n, h->lat[h->parity ^ 1]);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return II_LBM_EDEVICE;
        h->parity ^= 1;
    }
    return II_LBM_OK;
}

int ii_lbm3_set_distrib(ii_lbm3_handle* h, const double* f)
{
    if (!h || !f) return II_LBM_EINVAL;
    const Box& b = h->b;
    const long long n = (long long)b.nx * b.ny * b.nz;
    double* df = nullptr;
    hipError_t e = dmalloc(h, &df, (size_t)kQ * n * sizeof(double));
    if (e == hipSuccess) e = hipMemcpyAsync(df, f, (size_t)kQ * n * sizeof(double), hipMemcpyHostToDevice, h->stream);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_set3, dim3(1024), dim3(256), 0, h->stream, b, df, h->lat[h->parity]);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    else (void)hipStreamSynchronize(h->stream);
    dfree(h, df);
    return fail3(e);
}

int ii_lbm3_fields(ii_lbm3_handle* h, double* out)
{
    if (!h || !out) return II_LBM_EINVAL;
    const Box& b = h->b;
    const long long n = (long long)b.nx * b.ny * b.nz;
    double* d = nullptr;
    hipError_t e = dmalloc(h, &d, (size_t)4 * n * sizeof(double));
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_fields3, dim3(1024), dim3(256), 0, h->stream, b, h->lat[h->parity], d);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipMemcpyAsync(out, d, (size_t)4 * n * sizeof(double), hipMemcpyDeviceToHost, h->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    else (void)hipStreamSynchronize(h->stream);
    dfree(h, d);
    return fail3(e);
}

int ii_lbm3_set_timing(ii_lbm3_handle* h, int32_t enable)
{
    if (!h) return II_LBM_EINVAL;
    if (hipStreamSynchronize(h->stream) != hipSuccess) return II_LBM_EDEVICE;
    h->timing = enable != 0;
    h->ev_used = 0;
    return II_LBM_OK;
}

int ii_lbm3_get_timing(ii_lbm3_handle* h, double* ms, int64_t* launches)
{
    if (!h || !ms || !launches) return II_LBM_EINVAL;
    if (hipStreamSynchronize(h->stream) != hipSuccess) return II_LBM_EDEVICE;
    double total = 0.0;
    for (int k = 0; k + 1 < h->ev_used; k += 2) {
        float t = 0.f;
        if (hipEventElapsedTime(&t, h->ev[k], h->ev[k + 1]) != hipSuccess) return II_LBM_EDEVICE;
        total += t;
    }
    *ms = total;
    *launches = h->ev_used / 2;
    return II_LBM_OK;
}

int ii_lbm3_sweep_bytes(ii_lbm3_handle* h, double* bytes)
{
    if (!h || !bytes) return II_LBM_EINVAL;
    const double n = (double)h->b.nx * h->b.ny * h->b.nz;
    *bytes = n * (2.0 * kQ * 4.0 + ((h->b.ib || h->memb) ? 24.0 : 0.0));
    return II_LBM_OK;
}

int ii_lbm3_check_mesh(const ii_lbm3_problem* p, int32_t n_vert, const double* X, int32_t n_tri,
                       const int32_t* tri)
{
    if (!p || !X || !tri || n_vert < 4 || n_tri < 4 || n_vert > (1 << 20) || n_tri > (1 << 20))
        return II_LBM_EINVAL;
    if (p->force_mode != II_LBM_FORCE_II) return II_LBM_EINVAL;
    const int n[3] = {p->nx, p->ny, p->nz};
    std::vector<long long> S((size_t)3 * n_vert);
    for (int v = 0; v < n_vert; v++)
        for (int a = 0; a < 3; a++) {
            const double c = X[3 * v + a];
            if (!isfinite(c)) return II_LBM_EINVAL;
            if (!(c >= 2.0 && c <= n[a] - 3.0)) return II_LBM_EGEOMETRY;
            S[3 * v + a] = snap_2m16(c);
        }
    const long long lim = 4LL << 16;
    std::vector<unsigned long long> edges;
    edges.reserve((size_t)3 * n_tri);
    double vol = 0.0;
    for (int t = 0; t < n_tri; t++) {
        const int v[3] = {tri[3 * t], tri[3 * t + 1], tri[3 * t + 2]};
        for (int k = 0; k < 3; k++)
            if (v[k] < 0 || v[k] >= n_vert) return II_LBM_EINVAL;
        if (v[0] == v[1] || v[1] == v[2] || v[0] == v[2]) return II_LBM_EINVAL;
        for (int k = 0; k < 3; k++) {
            const long long* a = &S[3 * v[k]];
            const long long* c = &S[3 * v[(k + 1) % 3]];
            double len2 = 0.0;
            for (int j = 0; j < 3; j++) len2 += (double)(c[j] - a[j]) * (double)(c[j] - a[j]);
            if (len2 > (double)lim * (double)lim) return II_LBM_EGEOMETRY;
            edges.push_back((unsigned long long)v[k] * (unsigned long long)n_vert + (unsigned long long)v[(k + 1) % 3]);
        }
        const long long* A = &S[3 * v[0]];
        const long long* B = &S[3 * v[1]];
        const long long* C = &S[3 * v[2]];
        const long long ux = B[0] - A[0], uy = B[1] - A[1], uz = B[2] - A[2];
        const long long wx = C[0] - A[0], wy = C[1] - A[1], wz = C[2] - A[2];
        const long long cx = uy * wz - uz * wy, cy = uz * wx - ux * wz, cz = ux * wy - uy * wx;
        if (!cx && !cy && !cz) return II_LBM_EGEOMETRY;          // degenerate triangle
        // signed volume of the tetrahedron (vertex 0, A, B, C), in lu^3 * 6
        const double* X0 = X;
        double a0[3], b0[3], c0[3];
        for (int j = 0; j < 3; j++) {
            a0[j] = X[3 * v[0] + j] - X0[j]; b0[j] = X[3 * v[1] + j] - X0[j]; c0[j] = X[3 * v[2] + j] - X0[j];
        }
        vol += a0[0] * (b0[1] * c0[2] - b0[2] * c0[1]) - a0[1] * (b0[0] * c0[2] - b0[2] * c0[0]) +
               a0[2] * (b0[0] * c0[1] - b0[1] * c0[0]);
    }
    // closed and consistently oriented: every directed edge once, and its reverse once
    std::vector<unsigned long long> sorted(edges);
    std::sort(sorted.begin(), sorted.end());
    for (size_t k = 1; k < sorted.size(); k++)
        if (sorted[k] == sorted[k - 1]) return II_LBM_EGEOMETRY;
    for (unsigned long long e : sorted) {
        const unsigned long long r = (e % (unsigned long long)n_vert) * (unsigned long long)n_vert +
                                     e / (unsigned long long)n_vert;
        if (!std::binary_search(sorted.begin(), sorted.end(), r)) return II_LBM_EGEOMETRY;
    }
    if (!(vol > 0.0)) return II_LBM_EGEOMETRY;                   // outward orientation
    return II_LBM_OK;
}

int ii_lbm3_set_mesh(ii_lbm3_handle* h, int32_t n_vert, const double* X, int32_t n_tri, const int32_t* tri,
                     const double* jump_p, int64_t* n_links)
{
    if (!h) return II_LBM_EINVAL;
    if (hipStreamSynchronize(h->stream) != hipSuccess) return II_LBM_EDEVICE;
    free_mesh(h);
    if (n_links) *n_links = 0;
    if (n_vert != 0 || n_tri != 0) free_membrane(h);             // one surface at a time
    if (n_vert == 0 && n_tri == 0) return II_LBM_OK;            // surface removed
    const int rc = ii_lbm3_check_mesh(&h->prob, n_vert, X, n_tri, tri);
    if (rc != II_LBM_OK) return rc;
    if (!jump_p) return II_LBM_EINVAL;
    for (int v = 0; v < n_vert; v++)
        if (!isfinite(jump_p[v])) return II_LBM_EINVAL;
    std::vector<long long> S((size_t)3 * n_vert);
    for (size_t k = 0; k < S.size(); k++) S[k] = snap_2m16(X[k]);
    const long long cap = 64LL * n_tri + 4096;
    hipError_t e = dmalloc(h, &h->mesh_S, S.size() * sizeof(long long));
    if (e == hipSuccess) e = dmalloc(h, &h->mesh_tri, (size_t)3 * n_tri * sizeof(int));
    if (e == hipSuccess) e = dmalloc(h, &h->mesh_pv, (size_t)n_vert * sizeof(double));
    if (e == hipSuccess) e = dmalloc(h, &h->mesh_rec, (size_t)cap * sizeof(MeshRec3));
    if (e == hipSuccess) e = dmalloc(h, &h->mesh_count, sizeof(int));
    if (e == hipSuccess)
        e = hipMemcpyAsync(h->mesh_S, S.data(), S.size() * sizeof(long long), hipMemcpyHostToDevice, h->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(h->mesh_tri, tri, (size_t)3 * n_tri * sizeof(int), hipMemcpyHostToDevice, h->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(h->mesh_pv, jump_p, (size_t)n_vert * sizeof(double), hipMemcpyHostToDevice, h->stream);
    if (e == hipSuccess) e = hipMemsetAsync(h->mesh_count, 0, sizeof(int), h->stream);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_mesh_links3, dim3((n_tri + kMeshWaves - 1) / kMeshWaves), dim3(256), 0, h->stream,
                           h->mesh_S, h->mesh_tri, h->mesh_pv, n_tri, h->mesh_rec, (int)cap, h->mesh_count,
                           (const int*)nullptr);
        e = hipGetLastError();
    }
    int count = 0;
    if (e == hipSuccess) e = hipMemcpyAsync(&count, h->mesh_count, sizeof(int), hipMemcpyDeviceToHost, h->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    if (e != hipSuccess) {
        free_mesh(h);
        return II_LBM_EDEVICE;
    }
    if (count > cap) {
        free_mesh(h);
        return II_LBM_ECAPACITY;
    }
    // The per-step apply list: target offsets sorted, links that hit the same
    // population (a link crossing twice) merged in a fixed order.
    std::vector<MeshRec3> r(count);
    e = hipMemcpyAsync(r.data(), h->mesh_rec, r.size() * sizeof(MeshRec3), hipMemcpyDeviceToHost, h->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    const Box& b = h->b;
    std::vector<std::pair<long long, long long>> key(count);   // (offset, record's own order key)
    for (int k = 0; k < count; k++) {
        const MeshRec3& q = r[k];
        if (q.x < 0 || q.x >= b.nx || q.y < 0 || q.y >= b.ny || q.z < 0 || q.z >= b.nz || q.dir < 1 ||
            q.dir >= kQ || q.tri < 0 || q.tri >= n_tri) {
            free_mesh(h);
            return II_LBM_EDEVICE;
        }
        key[k] = {q.dir * b.plane + ((long long)q.z * b.ny + q.y) * b.pitch + q.x,
                  (long long)q.tri * 32 + q.dir};
        key[k].second = key[k].second * (1LL << 31) + k;     // ties: triangle, then slot
    }
    std::vector<int> order(count);
    for (int k = 0; k < count; k++) order[k] = k;
    std::sort(order.begin(), order.end(), [&](int a, int c) { return key[a] < key[c]; });
    std::vector<long long> off;
    std::vector<float> delta;
    for (int k = 0; k < count; k++) {
        const int j = order[k];
        if (!off.empty() && off.back() == key[j].first)
            delta.back() += r[j].delta;
        else {
            off.push_back(key[j].first);
            delta.push_back(r[j].delta);
        }
    }
    if (e == hipSuccess && !off.empty()) e = dmalloc(h, &h->apply_off, off.size() * sizeof(long long));
    if (e == hipSuccess && !off.empty()) e = dmalloc(h, &h->apply_delta, delta.size() * sizeof(float));
    if (e == hipSuccess && !off.empty())
        e = hipMemcpyAsync(h->apply_off, off.data(), off.size() * sizeof(long long), hipMemcpyHostToDevice,
                           h->stream);
    if (e == hipSuccess && !off.empty())
        e = hipMemcpyAsync(h->apply_delta, delta.data(), delta.size() * sizeof(float), hipMemcpyHostToDevice,
                           h->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    if (e != hipSuccess) {
        free_mesh(h);
        return II_LBM_EDEVICE;
    }
    h->mesh_links = count;
    h->apply_n = (int)off.size();
    if (n_links) *n_links = count;
    return II_LBM_OK;
}

static int set_surface(ii_lbm3_handle* h, int32_t n_vert, const double* X, int32_t n_tri, const int32_t* tri,
                       double gamma, int law)
{
    if (!h) return II_LBM_EINVAL;
    if (hipStreamSynchronize(h->stream) != hipSuccess) return II_LBM_EDEVICE;
    free_membrane(h);
    if (n_vert == 0 && n_tri == 0) return II_LBM_OK;             // membrane removed
    // the membrane's sweep reads the force field and carries no level-set jumps
    if (h->b.sphere || !isfinite(gamma) || gamma < 0.0) return II_LBM_EINVAL;
    ii_lbm3_problem geo = h->prob;
    geo.force_mode = II_LBM_FORCE_II;                             // the geometry rules only
    const int rc = ii_lbm3_check_mesh(&geo, n_vert, X, n_tri, tri);
    if (rc != II_LBM_OK) return rc;
    free_mesh(h);                                                 // one surface at a time
    std::vector<int> off(n_vert + 1, 0), vt((size_t)3 * n_tri);
    for (int t = 0; t < n_tri; t++)
        for (int k = 0; k < 3; k++) off[tri[3 * t + k] + 1]++;
    for (int v = 0; v < n_vert; v++) off[v + 1] += off[v];
    std::vector<int> fill(off.begin(), off.end() - 1);
    for (int t = 0; t < n_tri; t++)                               // ascending triangle order per vertex
        for (int k = 0; k < 3; k++) vt[fill[tri[3 * t + k]]++] = t;
    const long long n = (long long)h->b.nx * h->b.ny * h->b.nz;
    const int cap = 64 * n_tri + 4096;
    hipError_t e = hipSuccess;
    if (!h->g) e = dmalloc(h, &h->g, (size_t)3 * n * sizeof(long long));
    // the force field starts at zero; each step then clears what it spread
    if (e == hipSuccess) e = hipMemsetAsync(h->g, 0, (size_t)3 * n * sizeof(long long), h->stream);
    if (e == hipSuccess) e = dmalloc(h, &h->memb_X, (size_t)3 * n_vert * sizeof(double));
    if (e == hipSuccess) e = dmalloc(h, &h->memb_U, (size_t)3 * n_vert * sizeof(double));
    if (e == hipSuccess) e = dmalloc(h, &h->memb_jp, (size_t)n_vert * sizeof(double));
    if (e == hipSuccess) e = dmalloc(h, &h->memb_Gt, (size_t)3 * n_vert * sizeof(double));
    if (e == hipSuccess) e = dmalloc(h, &h->memb_G, (size_t)3 * n_vert * sizeof(double));
    if (e == hipSuccess) e = hipMemsetAsync(h->memb_G, 0, (size_t)3 * n_vert * sizeof(double), h->stream);
    if (e == hipSuccess) e = dmalloc(h, &h->memb_S, (size_t)3 * n_vert * sizeof(long long));
    if (e == hipSuccess) e = dmalloc(h, &h->memb_tri, (size_t)3 * n_tri * sizeof(int));
    if (e == hipSuccess) e = dmalloc(h, &h->memb_vt_off, (size_t)(n_vert + 1) * sizeof(int));
    if (e == hipSuccess) e = dmalloc(h, &h->memb_vt, vt.size() * sizeof(int));
    if (e == hipSuccess) e = dmalloc(h, &h->memb_rec, (size_t)cap * sizeof(MeshRec3));
    if (e == hipSuccess) e = dmalloc(h, &h->memb_count, sizeof(int));
    if (e == hipSuccess) e = dmalloc(h, &h->memb_err, sizeof(int));
    // per-target sums: twice as many entries as records can be (a table
    // sized for the usual 7 cut links per triangle was slower: its atomics
    // share more cache lines)
    int hbits = 1;
    while ((1LL << hbits) < 2LL * cap) hbits++;
    const size_t hn = (size_t)1 << hbits;
    if (e == hipSuccess) e = dmalloc(h, &h->memb_hkeys, hn * sizeof(unsigned long long));
    if (e == hipSuccess) e = dmalloc(h, &h->memb_hsums, hn * sizeof(long long));
    if (e == hipSuccess) e = dmalloc(h, &h->memb_used, (size_t)cap * sizeof(int));
    if (e == hipSuccess) e = dmalloc(h, &h->memb_nused, sizeof(int));
    if (e == hipSuccess) e = hipMemsetAsync(h->memb_hkeys, 0xff, hn * sizeof(unsigned long long), h->stream);
    if (e == hipSuccess) e = hipMemsetAsync(h->memb_hsums, 0, hn * sizeof(long long), h->stream);
    if (e == hipSuccess) e = hipMemsetAsync(h->memb_nused, 0, sizeof(int), h->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(h->memb_X, X, (size_t)3 * n_vert * sizeof(double), hipMemcpyHostToDevice, h->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(h->memb_tri, tri, (size_t)3 * n_tri * sizeof(int), hipMemcpyHostToDevice, h->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(h->memb_vt_off, off.data(), off.size() * sizeof(int), hipMemcpyHostToDevice, h->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(h->memb_vt, vt.data(), vt.size() * sizeof(int), hipMemcpyHostToDevice, h->stream);
    if (e == hipSuccess) e = hipMemsetAsync(h->memb_U, 0, (size_t)3 * n_vert * sizeof(double), h->stream);
    if (e == hipSuccess) e = hipMemsetAsync(h->memb_count, 0, sizeof(int), h->stream);
    if (e == hipSuccess) e = hipMemsetAsync(h->memb_err, 0, sizeof(int), h->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    if (e != hipSuccess) {
        free_membrane(h);
        return II_LBM_EDEVICE;
    }
    h->memb = true;
    h->memb_nv = n_vert;
    h->memb_nt = n_tri;
    h->memb_cap = cap;
    h->memb_hbits = hbits;
    h->memb_gamma = gamma;
    h->memb_law = law;
    return II_LBM_OK;
}

int ii_lbm3_set_membrane(ii_lbm3_handle* h, int32_t n_vert, const double* X, int32_t n_tri, const int32_t* tri,
                         double gamma)
{
    if (!h) return II_LBM_EINVAL;
    return set_surface(h, n_vert, X, n_tri, tri, gamma, h->prob.force_mode == II_LBM_FORCE_IB ? 2 : 0);
}

int ii_lbm3_set_rigid_surface(ii_lbm3_handle* h, int32_t n_vert, const double* X, int32_t n_tri,
                              const int32_t* tri)
{
    if (!h) return II_LBM_EINVAL;
    if (h->prob.force_mode != II_LBM_FORCE_II) return II_LBM_EINVAL;
    return set_surface(h, n_vert, X, n_tri, tri, 0.0, 1);
}

int ii_lbm3_set_free_sphere(ii_lbm3_handle* h, int32_t n_vert, const double* X, int32_t n_tri,
                            const int32_t* tri, const double* center, double radius, double rho_star,
                            const double* U0, const double* W0)
{
    if (!h || !center || !U0 || !W0) return II_LBM_EINVAL;
    if (h->prob.force_mode != II_LBM_FORCE_II) return II_LBM_EINVAL;
    if (!(radius > 0.0) || !isfinite(radius) || !(rho_star > 0.0) || !isfinite(rho_star)) return II_LBM_EINVAL;
    for (int k = 0; k < 3; k++)
        if (!isfinite(center[k]) || !isfinite(U0[k]) || !isfinite(W0[k])) return II_LBM_EINVAL;
    int rc = set_surface(h, n_vert, X, n_tri, tri, 0.0, 3);
    if (rc != II_LBM_OK) return rc;
    Body3 b;
    memset(&b, 0, sizeof b);
    for (int k = 0; k < 3; k++) {
        b.c[k] = center[k];
        b.U[k] = b.Up[k] = U0[k];
        b.W[k] = b.Wp[k] = W0[k];
    }
    hipError_t e = dmalloc(h, &h->body3, sizeof(Body3));
    if (e == hipSuccess) e = hipMemcpyAsync(h->body3, &b, sizeof b, hipMemcpyHostToDevice, h->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    if (e != hipSuccess) {
        free_membrane(h);
        return II_LBM_EDEVICE;
    }
    h->body3_radius = radius;
    h->body3_rho = rho_star;
    return II_LBM_OK;
}

int ii_lbm3_body(ii_lbm3_handle* h, double* out)
{
    if (!h || !out) return II_LBM_EINVAL;
    if (!h->memb || h->memb_law != 3 || !h->body3) return II_LBM_ESTATE;
    Body3 b;
    int err = 0;
    hipError_t e = hipMemcpyAsync(&b, h->body3, sizeof b, hipMemcpyDeviceToHost, h->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(&err, h->memb_err, sizeof(int), hipMemcpyDeviceToHost, h->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    if (e != hipSuccess) return II_LBM_EDEVICE;
    const double* src[9] = {b.c, b.U, b.a, b.W, b.wd, b.Up, b.Wp, b.F, b.T};
    for (int q = 0; q < 9; q++)
        for (int k = 0; k < 3; k++) out[3 * q + k] = src[q][k];
    if (err & 2) return II_LBM_ECAPACITY;
    if (err & 1) return II_LBM_EGEOMETRY;
    return II_LBM_OK;
}

int ii_lbm3_surface_force(ii_lbm3_handle* h, double* F)
{
    if (!h || !F) return II_LBM_EINVAL;
    if (!h->memb) return II_LBM_ESTATE;
    std::vector<double> G((size_t)3 * h->memb_nv);
    int err = 0;
    hipError_t e = hipMemcpyAsync(G.data(), h->memb_G, G.size() * sizeof(double), hipMemcpyDeviceToHost, h->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(&err, h->memb_err, sizeof(int), hipMemcpyDeviceToHost, h->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    if (e != hipSuccess) return II_LBM_EDEVICE;
    F[0] = F[1] = F[2] = 0.0;
    for (int v = 0; v < h->memb_nv; v++)
        for (int k = 0; k < 3; k++) F[k] -= G[3 * v + k];
    if (err & 2) return II_LBM_ECAPACITY;
    if (err & 1) return II_LBM_EGEOMETRY;
    return II_LBM_OK;
}

int ii_lbm3_membrane(ii_lbm3_handle* h, double* X, double* U)
{
    if (!h) return II_LBM_EINVAL;
    if (!h->memb) return II_LBM_ESTATE;
    int err = 0;
    hipError_t e = hipMemcpyAsync(&err, h->memb_err, sizeof(int), hipMemcpyDeviceToHost, h->stream);
    if (e == hipSuccess && X)
        e = hipMemcpyAsync(X, h->memb_X, (size_t)3 * h->memb_nv * sizeof(double), hipMemcpyDeviceToHost, h->stream);
    if (e == hipSuccess && U)
        e = hipMemcpyAsync(U, h->memb_U, (size_t)3 * h->memb_nv * sizeof(double), hipMemcpyDeviceToHost, h->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    if (e != hipSuccess) return II_LBM_EDEVICE;
    if (err & 2) return II_LBM_ECAPACITY;
    if (err & 1) return II_LBM_EGEOMETRY;
    return II_LBM_OK;
}

int ii_lbm3_mesh_links(ii_lbm3_handle* h, int64_t cap, int32_t* rec, double* jp, int64_t* n_links)
{
    if (!h || !n_links || cap < 0 || (cap > 0 && (!rec || !jp))) return II_LBM_EINVAL;
    *n_links = h->mesh_links;
    if (h->mesh_links == 0) return II_LBM_OK;
    if (cap < h->mesh_links) return II_LBM_ECAPACITY;
    std::vector<MeshRec3> r(h->mesh_links);
    hipError_t e = hipMemcpyAsync(r.data(), h->mesh_rec, r.size() * sizeof(MeshRec3), hipMemcpyDeviceToHost,
                                  h->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    if (e != hipSuccess) return II_LBM_EDEVICE;
    for (size_t k = 0; k < r.size(); k++) {
        int32_t* o = rec + 6 * k;
        o[0] = r[k].x; o[1] = r[k].y; o[2] = r[k].z; o[3] = r[k].dir; o[4] = r[k].sigma; o[5] = r[k].tri;
        jp[k] = r[k].jp;
    }
    return II_LBM_OK;
}

int ii_lbm3_destroy(ii_lbm3_handle* h)
{
    if (!h) return II_LBM_EINVAL;
    (void)hipStreamSynchronize(h->stream);
    free_mesh(h);
    free_membrane(h);
    for (auto& p : h->lat) dfree(h, p);
    dfree(h, h->g);
    for (auto& ev : h->ev) (void)hipEventDestroy(ev);
    delete h;
    return II_LBM_OK;
}

}  // extern "C"
