// Interface kernels of one II-LBM step (compiled without FP contraction so
// that the FP64 geometry is evaluated exactly as written):
//   k_markers  one thread per marker: interpolated velocity U^n, force G^n,
//              outward normal, |dX/ds|, [[p]] and the tangential part; the new
//              position X^{n+1}; binning of chord (k, k+1) into 16x16 tiles.
//   k_tiles    one block per tile that holds chords: spreads the tangential
//              force onto its nodes, finds every cut link leaving its nodes
//              with exact integer predicates, adds the force term and the
//              jumps to the stored post-collision populations in one
//              read-modify-write, and compacts the cut-link records.
#include "common.hpp"

namespace iilbm {

constexpr double kCs2 = 1.0 / 3.0;

// Peskin's four-point regularized delta (cited in Sec. 2.1.2), one axis.
__device__ __forceinline__ double peskin(double r)
{
    const double a = fabs(r);
    if (a <= 1.0) return (3.0 - 2.0 * a + sqrt(1.0 + 4.0 * a - 4.0 * a * a)) * 0.125;
    if (a <= 2.0) return (5.0 - 2.0 * a - sqrt(-7.0 + 12.0 * a - 4.0 * a * a)) * 0.125;
    return 0.0;
}

__device__ __forceinline__ int wrap_or_clamp(int v, int n, int periodic)
{
    if (periodic) return ((v % n) + n) % n;
    return v < 0 ? 0 : (v >= n ? n - 1 : v);
}

// ---------------------------------------------------------------------------
// Markers.
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(256) void k_markers(InstDev I, DevPtrs P, const T* __restrict__ A,
                                                 int parity)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k == 0) {
        // counters of the other parity were consumed by the previous step
        P.act_count[2 * I.inst + (parity ^ 1)] = 0;
        P.rec_count[2 * I.inst + (parity ^ 1)] = 0;
    }
    if (k >= I.n_markers) return;
    const int N = I.n_markers;
    const double2* X = P.X[parity] + I.mk_off;
    double2* Xn = P.X[parity ^ 1] + I.mk_off;
    const double2 Xk = X[k];
    const int km = (k + N - 1) % N, kp = (k + 1) % N;
    const double2 Xm = X[km], Xp = X[kp];
    if (!(Xk.x >= 0.0 && Xk.x < (double)I.nx && Xk.y >= 0.0 && Xk.y < (double)I.ny)) {
        // non-finite or outside the lattice: keep the marker, flag the handle
        atomicOr(&P.err[I.inst], isfinite(Xk.x) && isfinite(Xk.y) ? (int)kErrGeometry
                                                                  : (int)kErrUnstable);
        const int m = I.mk_off + k;
        P.U[m] = make_double2(0.0, 0.0);
        P.G[m] = make_double2(0.0, 0.0);
        P.Gt[m] = make_double2(0.0, 0.0);
        P.jp[m] = 0.0;
        Xn[k] = Xk;
        return;
    }

    // U_k = sum_x u^n(x) delta_h(x - X_k) (Sec. 2.2.2, Eq. (20)); u^n from the
    // pre-collision f^n, summed in FP64 from the stored deviations.
    double us = 0.0, vs = 0.0;
    const int fx = (int)floor(Xk.x), fy = (int)floor(Xk.y);
    for (int y = fy - 1; y <= fy + 2; y++)
        for (int x = fx - 1; x <= fx + 2; x++) {
            const double w = peskin((double)x - Xk.x) * peskin((double)y - Xk.y);
            if (w == 0.0) continue;
            float d[9];
            gather<T>(I, A, wrap_or_clamp(x, I.nx, I.px), wrap_or_clamp(y, I.ny, I.py), d);
            double u = 0.0, v = 0.0;
#pragma unroll
            for (int i = 1; i < 9; i++) {
                u += (double)EX[i] * (double)d[i];
                v += (double)EY[i] * (double)d[i];
            }
            us += u * w;
            vs += v * w;
        }

    double gx, gy, nx_, ny_, jac;
    if (I.iface == II_LBM_IF_MEMBRANE) {
        // spring force kappa (X_{k+1} - 2 X_k + X_{k-1}) / dX^2 (Sec. 2.2.2, Eq. (19))
        const double d2 = I.dX * I.dX;
        gx = I.kappa * (Xp.x - 2.0 * Xk.x + Xm.x) / d2;
        gy = I.kappa * (Xp.y - 2.0 * Xk.y + Xm.y) / d2;
        // outward normal of the counter-clockwise curve, from the central chord
        const double tx = Xp.x - Xm.x, ty = Xp.y - Xm.y;
        const double tl = sqrt(tx * tx + ty * ty);
        nx_ = ty / tl;
        ny_ = -tx / tl;
        // |dX/ds|: mean length of the two chords at the marker over Delta X
        const double lp = hypot(Xp.x - Xk.x, Xp.y - Xk.y);
        const double lm = hypot(Xk.x - Xm.x, Xk.y - Xm.y);
        jac = (lp + lm) / (2.0 * I.dX);
    } else {
        // direct forcing to U^D = 0 with eta = 1 (Sec. 2.2.2, Eq. (18));
        // |dX/ds| = 1 and the radial normal of the rigid circle (Sec. 3.1)
        gx = 0.0 - us;
        gy = 0.0 - vs;
        nx_ = (Xk.x - I.cx) / I.radius;
        ny_ = (Xk.y - I.cy) / I.radius;
        jac = 1.0;
    }
    // [[p]] = G.n / |dX/ds| (Sec. 3.1, Eq. (40)); G_par = G - (G.n) n (Eq. (46))
    const double gn = gx * nx_ + gy * ny_;
    const int m = I.mk_off + k;
    P.U[m] = make_double2(us, vs);
    P.G[m] = make_double2(gx, gy);
    P.jp[m] = gn / jac;
    P.Gt[m] = make_double2(gx - gn * nx_, gy - gn * ny_);

    // X^{n+1} = X^n + U^n (Sec. 2.2.2, Eq. (20)); a fixed body stays put.
    double2 Xnew = Xk;
    if (I.iface == II_LBM_IF_MEMBRANE) Xnew = make_double2(Xk.x + us, Xk.y + vs);
    Xn[k] = Xnew;
    if (!isfinite(us) || !isfinite(vs)) atomicOr(&P.err[I.inst], (int)kErrUnstable);
    if (!(Xnew.x >= 3.0 && Xnew.x <= (double)(I.nx - 4) && Xnew.y >= 3.0 &&
          Xnew.y <= (double)(I.ny - 4)))
        atomicOr(&P.err[I.inst], (int)kErrGeometry);

    // Bin chord (k, k+1) into every tile within 2.5 lu of it: those tiles hold
    // the nodes whose links it can cut and the support of marker k's delta.
    const double xmin = fmin(Xk.x, Xp.x) - 2.5, xmax = fmax(Xk.x, Xp.x) + 2.5;
    const double ymin = fmin(Xk.y, Xp.y) - 2.5, ymax = fmax(Xk.y, Xp.y) + 2.5;
    if (!(xmin == xmin) || !(ymin == ymin) || !(xmax == xmax) || !(ymax == ymax)) return;
    const int tx0 = max(0, (int)floor(fmax(xmin, 0.0) / kTile));
    const int tx1 = min(I.tiles_x - 1, (int)floor(fmin(xmax, (double)I.nx) / kTile));
    const int ty0 = max(0, (int)floor(fmax(ymin, 0.0) / kTile));
    const int ty1 = min(I.tiles_y - 1, (int)floor(fmin(ymax, (double)I.ny) / kTile));
    for (int ty = ty0; ty <= ty1; ty++)
        for (int tx = tx0; tx <= tx1; tx++) {
            const int t = ty * I.tiles_x + tx;
            const int gt = I.tile_off + t;
            const int pos = atomicAdd(&P.tile_count[gt], 1);
            if (pos < kTileCap)
                P.tile_list[(long long)gt * kTileCap + pos] = k;
            else
                atomicOr(&P.err[I.inst], (int)kErrCapacity);
            if (pos == 0) {
                const int a = atomicAdd(&P.act_count[2 * I.inst + parity], 1);
                if (a < I.act_cap)
                    P.act_list[I.act_off + a] = make_int2(I.inst, t);
                else
                    atomicOr(&P.err[I.inst], (int)kErrCapacity);
            }
        }
}

template <typename T>
static hipError_t markers_t(const InstDev& I, const DevPtrs& P, const void* A, int parity,
                            hipStream_t s)
{
    const int nb = (I.n_markers + 255) / 256;
    hipLaunchKernelGGL(k_markers<T>, dim3(nb), dim3(256), 0, s, I, P, (const T*)A, parity);
    return hipGetLastError();
}

hipError_t launch_markers(const InstDev& I, const DevPtrs& P, const void* A, int parity,
                          hipStream_t s)
{
    return I.storage == II_LBM_FP16 ? markers_t<_Float16>(I, P, A, parity, s)
                                    : markers_t<float>(I, P, A, parity, s);
}

// ---------------------------------------------------------------------------
// Exact link/chord crossing on the 2^-16 snapped grid.
// ---------------------------------------------------------------------------
__device__ __forceinline__ long long cross3(long long ax, long long ay, long long bx, long long by,
                                            long long cx, long long cy)
{
    return (bx - ax) * (cy - ay) - (by - ay) * (cx - ax);
}

// Side (+1 left / -1 right) of the lattice node shifted by (eps, eps^2)
// relative to the directed chord a->b; a zero orientation is decided by the
// shift, so the result is never zero.
__device__ __forceinline__ int node_side(long long ax, long long ay, long long bx, long long by,
                                         long long px, long long py)
{
    const long long o = cross3(ax, ay, bx, by, px, py);
    if (o > 0) return 1;
    if (o < 0) return -1;
    const long long dy = by - ay, dx = bx - ax;
    if (dy != 0) return dy > 0 ? -1 : 1;
    return dx > 0 ? 1 : -1;
}

// Side of chord end c relative to the link p->q, both link ends shifted by the
// same (eps, eps^2).
__device__ __forceinline__ int end_side(long long px, long long py, long long qx, long long qy,
                                        long long cx, long long cy)
{
    const long long o = cross3(px, py, qx, qy, cx, cy);
    if (o > 0) return 1;
    if (o < 0) return -1;
    const long long dy = qy - py, dx = qx - px;
    if (dy != 0) return dy > 0 ? 1 : -1;
    return dx > 0 ? -1 : 1;
}

// ---------------------------------------------------------------------------
// Tiles.
// ---------------------------------------------------------------------------
struct TileShared {
    int raw[kTileCap];
    int key[kTileCap];
    long long ax[kTileCap], ay[kTileCap], bx[kTileCap], by[kTileCap];
    int box[kTileCap][4];
    double jpa[kTileCap], jpb[kTileCap];
    double mx[kTileCap], my[kTileCap], gtx[kTileCap], gty[kTileCap];
    int cnt, base, tot;
    int woff[4];
};

template <typename T, int IFACE>
__global__ __launch_bounds__(256) void k_tiles(InstDev I, DevPtrs P, T* __restrict__ B,
                                               int parity, int records)
{
    __shared__ TileShared S;
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    const int N = I.n_markers;
    const double2* X = P.X[parity] + I.mk_off;
    const int nact = min(P.act_count[2 * I.inst + parity], I.act_cap);
    for (int a = blockIdx.x; a < nact; a += gridDim.x) {
        const int t = P.act_list[I.act_off + a].y;
        const int gt = I.tile_off + t;
        if (tid == 0) S.cnt = min(P.tile_count[gt], kTileCap);
        __syncthreads();
        const int c = S.cnt;
        if (tid < c) S.raw[tid] = P.tile_list[(long long)gt * kTileCap + tid];
        __syncthreads();
        if (tid == 0) P.tile_count[gt] = 0;  // ready for the next step
        // deterministic order: rank sort of the (distinct) chord ids
        if (tid < c) {
            const int key = S.raw[tid];
            int r = 0;
            for (int m = 0; m < c; m++) r += (S.raw[m] < key) ? 1 : 0;
            S.key[r] = key;
        }
        __syncthreads();
        if (tid < c) {
            const int k = S.key[tid], kp = (k + 1) % N;
            const double2 a0 = X[k], b0 = X[kp];
            const long long ax = (long long)rint(a0.x * kSnap), ay = (long long)rint(a0.y * kSnap);
            const long long bx = (long long)rint(b0.x * kSnap), by = (long long)rint(b0.y * kSnap);
            S.ax[tid] = ax; S.ay[tid] = ay; S.bx[tid] = bx; S.by[tid] = by;
            S.box[tid][0] = (int)(min(ax, bx) >> 16);
            S.box[tid][1] = (int)(-((-max(ax, bx)) >> 16));
            S.box[tid][2] = (int)(min(ay, by) >> 16);
            S.box[tid][3] = (int)(-((-max(ay, by)) >> 16));
            S.jpa[tid] = P.jp[I.mk_off + k];
            S.jpb[tid] = P.jp[I.mk_off + kp];
            S.mx[tid] = a0.x; S.my[tid] = a0.y;
            const double2 g = P.Gt[I.mk_off + k];
            S.gtx[tid] = g.x; S.gty[tid] = g.y;
        }
        __syncthreads();

        const int tx = t % I.tiles_x, ty = t / I.tiles_x;
        const int x = tx * kTile + (tid & (kTile - 1)), y = ty * kTile + tid / kTile;
        const bool valid = x < I.nx && y < I.ny;
        double gx = 0.0, gy = 0.0;
        double acc[9];
#pragma unroll
        for (int i = 0; i < 9; i++) acc[i] = 0.0;
        int ncross = 0;
        if (valid) {
            // tangential force g_par(x) = sum_k G_par,k delta_h(x - X_k) dX (Sec. 3.2, Eq. (46))
            for (int j = 0; j < c; j++) {
                const double rx = (double)x - S.mx[j];
                if (fabs(rx) >= 2.0) continue;
                const double ry = (double)y - S.my[j];
                if (fabs(ry) >= 2.0) continue;
                const double w = peskin(rx) * peskin(ry);
                gx += S.gtx[j] * w * I.dX;
                gy += S.gty[j] * w * I.dX;
            }
            // jumps sigma [[f_i]] = sigma w_i [[p]] / c_s^2 on every cut link
            // leaving (x, y) (Sec. 3.1, Eq. (32); Sec. 3.2, Eq. (47))
            if (IFACE == II_LBM_IF_MEMBRANE) {
                const long long px = (long long)x << 16, py = (long long)y << 16;
                for (int j = 0; j < c; j++) {
                    if (x + 1 < S.box[j][0] || x - 1 > S.box[j][1] || y + 1 < S.box[j][2] ||
                        y - 1 > S.box[j][3])
                        continue;
                    const long long ax = S.ax[j], ay = S.ay[j], bx = S.bx[j], by = S.by[j];
                    const int sp = node_side(ax, ay, bx, by, px, py);
#pragma unroll
                    for (int i = 1; i < 9; i++) {
                        const long long qx = (long long)(x + EX[i]) << 16;
                        const long long qy = (long long)(y + EY[i]) << 16;
                        if (node_side(ax, ay, bx, by, qx, qy) == sp) continue;
                        if (end_side(px, py, qx, qy, ax, ay) == end_side(px, py, qx, qy, bx, by))
                            continue;
                        const double oA = (double)cross3(px, py, qx, qy, ax, ay);
                        const double oB = (double)cross3(px, py, qx, qy, bx, by);
                        const double th = oA / (oA - oB);
                        const double jpc = (1.0 - th) * S.jpa[j] + th * S.jpb[j];
                        const double sg = sp > 0 ? 1.0 : -1.0;
                        acc[i] += sg * WD[i] * jpc / kCs2;
                        ncross++;
                    }
                }
            } else {
                const double R2 = I.radius * I.radius;
                const double phP =
                    ((double)x - I.cx) * ((double)x - I.cx) + ((double)y - I.cy) * ((double)y - I.cy) - R2;
#pragma unroll
                for (int i = 1; i < 9; i++) {
                    const double qxd = (double)(x + EX[i]), qyd = (double)(y + EY[i]);
                    const double phQ = (qxd - I.cx) * (qxd - I.cx) + (qyd - I.cy) * (qyd - I.cy) - R2;
                    const bool inP = phP < 0.0, inQ = phQ < 0.0;
                    if (inP == inQ) continue;
                    const double dx = (double)x - I.cx, dy = (double)y - I.cy;
                    const double ee = (double)(EX[i] * EX[i] + EY[i] * EY[i]);
                    const double de = dx * EX[i] + dy * EY[i];
                    const double dd = dx * dx + dy * dy - R2;
                    const double disc = sqrt(de * de - ee * dd);
                    const double q = inP ? (-de + disc) / ee : (-de - disc) / ee;
                    const double cxp = (double)x + q * EX[i] - I.cx, cyp = (double)y + q * EY[i] - I.cy;
                    double ang = atan2(cyp, cxp);
                    if (ang < 0.0) ang += 2.0 * M_PI;
                    const double sN = ang * N / (2.0 * M_PI);
                    int k = (sN >= 0.0 && sN < (double)N) ? (int)floor(sN) : 0;
                    const double th = sN - k;
                    const double jpc = (1.0 - th) * P.jp[I.mk_off + k] + th * P.jp[I.mk_off + (k + 1) % N];
                    acc[i] += (inP ? 1.0 : -1.0) * WD[i] * jpc / kCs2;
                    ncross++;
                }
            }
        }

        // Record compaction: block-wide exclusive prefix sum of the per-node
        // crossing counts (wavefront scan + four wave totals), one atomic per
        // tile for the base of its slice.
        int v = ncross;
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            const int o = __shfl_up(v, off, 64);
            if (lane >= off) v += o;
        }
        if (lane == 63) S.woff[wid] = v;
        __syncthreads();
        if (tid == 0) {
            int tot = 0;
            for (int w = 0; w < 4; w++) {
                const int cw = S.woff[w];
                S.woff[w] = tot;
                tot += cw;
            }
            S.tot = tot;
            S.base = (records && tot > 0) ? atomicAdd(&P.rec_count[2 * I.inst + parity], tot) : 0;
        }
        __syncthreads();
        if (records && S.tot > 0 && valid && ncross > 0) {
            int o = S.base + S.woff[wid] + (v - ncross);
            if (IFACE == II_LBM_IF_MEMBRANE) {
                const long long px = (long long)x << 16, py = (long long)y << 16;
                for (int j = 0; j < c; j++) {
                    if (x + 1 < S.box[j][0] || x - 1 > S.box[j][1] || y + 1 < S.box[j][2] ||
                        y - 1 > S.box[j][3])
                        continue;
                    const long long ax = S.ax[j], ay = S.ay[j], bx = S.bx[j], by = S.by[j];
                    const int sp = node_side(ax, ay, bx, by, px, py);
                    for (int i = 1; i < 9; i++) {
                        const long long qx = (long long)(x + EX[i]) << 16;
                        const long long qy = (long long)(y + EY[i]) << 16;
                        if (node_side(ax, ay, bx, by, qx, qy) == sp) continue;
                        if (end_side(px, py, qx, qy, ax, ay) == end_side(px, py, qx, qy, bx, by))
                            continue;
                        const double oP = (double)cross3(ax, ay, bx, by, px, py);
                        const double oQ = (double)cross3(ax, ay, bx, by, qx, qy);
                        const double oA = (double)cross3(px, py, qx, qy, ax, ay);
                        const double oB = (double)cross3(px, py, qx, qy, bx, by);
                        const double th = oA / (oA - oB);
                        if (o < I.rec_cap) {
                            ii_lbm_link r;
                            r.x = x; r.y = y; r.dir = i; r.sigma = sp > 0 ? 1 : -1;
                            r.seg = S.key[j]; r.inst = I.inst;
                            r.q = oP / (oP - oQ); r.theta = th;
                            r.jp = (1.0 - th) * S.jpa[j] + th * S.jpb[j];
                            P.rec[I.rec_off + o] = r;
                        } else {
                            atomicOr(&P.err[I.inst], (int)kErrRecords);
                        }
                        o++;
                    }
                }
            } else {
                const double R2 = I.radius * I.radius;
                for (int i = 1; i < 9; i++) {
                    const double phP = ((double)x - I.cx) * ((double)x - I.cx) +
                                       ((double)y - I.cy) * ((double)y - I.cy) - R2;
                    const double qxd = (double)(x + EX[i]), qyd = (double)(y + EY[i]);
                    const double phQ = (qxd - I.cx) * (qxd - I.cx) + (qyd - I.cy) * (qyd - I.cy) - R2;
                    const bool inP = phP < 0.0, inQ = phQ < 0.0;
                    if (inP == inQ) continue;
                    const double dx = (double)x - I.cx, dy = (double)y - I.cy;
                    const double ee = (double)(EX[i] * EX[i] + EY[i] * EY[i]);
                    const double de = dx * EX[i] + dy * EY[i];
                    const double dd = dx * dx + dy * dy - R2;
                    const double disc = sqrt(de * de - ee * dd);
                    const double q = inP ? (-de + disc) / ee : (-de - disc) / ee;
                    const double cxp = (double)x + q * EX[i] - I.cx, cyp = (double)y + q * EY[i] - I.cy;
                    double ang = atan2(cyp, cxp);
                    if (ang < 0.0) ang += 2.0 * M_PI;
                    const double sN = ang * N / (2.0 * M_PI);
                    int k = (sN >= 0.0 && sN < (double)N) ? (int)floor(sN) : 0;
                    const double th = sN - k;
                    if (o < I.rec_cap) {
                        ii_lbm_link r;
                        r.x = x; r.y = y; r.dir = i; r.sigma = inP ? 1 : -1;
                        r.seg = k; r.inst = I.inst;
                        r.q = q; r.theta = th;
                        r.jp = (1.0 - th) * P.jp[I.mk_off + k] + th * P.jp[I.mk_off + (k + 1) % N];
                        P.rec[I.rec_off + o] = r;
                    } else {
                        atomicOr(&P.err[I.inst], (int)kErrRecords);
                    }
                    o++;
                }
            }
        }

        // One read-modify-write per corrected population: force term of the
        // tangential force plus the jumps of the links this node sends.
        if (valid) {
            T* base = B + I.lat_off + (long long)y * I.pitch + x;
#pragma unroll
            for (int i = 1; i < 9; i++) {
                const double delta =
                    3.0 * WD[i] * ((double)EX[i] * gx + (double)EY[i] * gy) + acc[i];
                if (delta != 0.0) {
                    T* pp = base + i * I.plane;
                    Store<T>::st(pp, Store<T>::ld(pp, I.scale) + (float)delta, I.inv_scale);
                }
            }
        }
        __syncthreads();
    }
}

template <typename T>
static hipError_t tiles_t(const InstDev& I, const DevPtrs& P, void* B, int parity, int records,
                          hipStream_t s)
{
    const int nb = max(1, min(I.act_cap, 2048));
    if (I.iface == II_LBM_IF_MEMBRANE)
        hipLaunchKernelGGL((k_tiles<T, II_LBM_IF_MEMBRANE>), dim3(nb), dim3(256), 0, s, I, P,
                           (T*)B, parity, records);
    else
        hipLaunchKernelGGL((k_tiles<T, II_LBM_IF_RIGID>), dim3(nb), dim3(256), 0, s, I, P, (T*)B,
                           parity, records);
    return hipGetLastError();
}

hipError_t launch_tiles(const InstDev& I, const DevPtrs& P, void* B, int parity, int records,
                        hipStream_t s)
{
    return I.storage == II_LBM_FP16 ? tiles_t<_Float16>(I, P, B, parity, records, s)
                                    : tiles_t<float>(I, P, B, parity, records, s);
}

}  // namespace iilbm
