// Dense lattice kernels: the fused pull-stream + collide sweep (the hot loop,
// nine loads and nine stores per node), the field readout, state set-up and
// the FP64 reductions for diagnostics.
#include "common.hpp"

namespace iilbm {

// One time step of the bulk: gather f^n at (x, y) (pulled populations that
// already carry the previous step's jumps and force; extrapolated on bounded
// sides), collide (SRT or MRT) with the uniform body force and this step's
// interface corrections (tangential force term and jumps of the links this
// node sends, prepared per 16x16 tile by the interface kernel) folded into
// the relaxation increment, and store the result at (x, y).  With FP64
// collision arithmetic every stored value is rounded exactly once; with FP32
// arithmetic d takes one rounding and the increment a few at its own, finer,
// scale.
// GUO: Guo's force term of the whole Eulerian force (the body force plus the
// spread force the tile's slot holds in its last two planes); the slot's
// population planes then hold the jumps alone.
template <typename T, typename M, int COLL, bool BOUNDED, bool GUO>
__device__ __forceinline__ void sweep_node(const InstDev& I, const T* __restrict__ A,
                                           T* __restrict__ B, int x, int y,
                                           const int* __restrict__ tile_slot,
                                           const float* __restrict__ corr,
                                           const unsigned long long* __restrict__ cmask)
{
    M d[9];
    if (BOUNDED && is_edge(I, x, y))
        nee<T, M>(I, A, x, y, d);
    else
        pull<T, M>(I, A, x, y, d);
    // this step's interface correction of the populations the node sends
    // (zero away from the interface); with Guo's term the slot's last two
    // planes add the spread force to the body force
    M xc[9];
#pragma unroll
    for (int i = 0; i < 9; i++) xc[i] = (M)0;
    M gx = (M)I.body[0], gy = (M)I.body[1];
    if (I.n_markers > 0) {
        const int slot = tile_slot[I.tile_off + (y / kTile) * I.tiles_x + (x / kTile)];
        const int node = (y % kTile) * kTile + (x % kTile);
        if (slot >= 0 && corr_present(cmask, slot, node)) {
            const float* c = corr + (long long)slot * kCorrPlanes * kTileNodes + node;
#pragma unroll
            for (int i = 1; i < 9; i++) xc[i] = (M)c[(i - 1) * kTileNodes];
            if constexpr (GUO) {
                gx += (M)c[8 * kTileNodes];
                gy += (M)c[9 * kTileNodes];
            }
        }
    }
    const M omega = sizeof(M) == 8 ? (M)I.omega_d : (M)I.omega;
    if constexpr (GUO) {
        if (COLL == II_LBM_SRT)
            collide_guo_srt<M>(d, omega, gx, gy, xc);
        else
            collide_guo_mrt<M>(d, I.s, gx, gy, xc);
    } else {
        if (COLL == II_LBM_SRT)
            collide_srt<M, sizeof(T) == 4>(d, omega, gx, gy, xc);
        else
            collide_mrt<M>(d, I.s, gx, gy, xc);
    }
    T* base = B + I.lat_off + (long long)y * I.pitch + x;
#pragma unroll
    for (int i = 0; i < 9; i++) Store<T>::st_stream(base + i * I.plane, (float)d[i], I.inv_scale);
}

template <typename T, typename M, int COLL, bool BOUNDED, int BX, bool GUO>
__global__ __launch_bounds__(BX) void k_sweep(InstDev I, const T* __restrict__ A,
                                              T* __restrict__ B, int bx_count,
                                              const int* __restrict__ tile_slot,
                                              const float* __restrict__ corr,
                                              const unsigned long long* __restrict__ cmask)
{
    // the interface pass of the next step may share the CUs: the sweep's
    // waves issue first
    __builtin_amdgcn_s_setprio(3);
    const int bx = blockIdx.x % bx_count, y = blockIdx.x / bx_count;
    const int x = bx * BX + threadIdx.x;
    if (x >= I.nx) return;
    sweep_node<T, M, COLL, BOUNDED, GUO>(I, A, B, x, y, tile_slot, corr, cmask);
}

// Batched: block b sweeps `UNIT` consecutive nodes (row-major) of one
// instance, from the work table; collision and boundary kind per instance.
template <typename T, typename M, int UNIT, bool GUO>
__global__ __launch_bounds__(UNIT) void k_sweep_batch(const InstDev* __restrict__ insts,
                                                      const int2* __restrict__ units,
                                                      const T* __restrict__ A, T* __restrict__ B,
                                                      const int* __restrict__ tile_slot,
                                                      const float* __restrict__ corr,
                                                      const unsigned long long* __restrict__ cmask)
{
    __builtin_amdgcn_s_setprio(3);
    const int2 u = units[blockIdx.x];
    if (u.x < 0) return;   // padding of the table
    const InstDev I = insts[u.x];
    const int r = u.y + threadIdx.x;
    if (r >= I.nx * I.ny) return;
    const int y = r / I.nx, x = r - y * I.nx;
    if (I.collision == II_LBM_SRT) {
        if (I.bounded)
            sweep_node<T, M, II_LBM_SRT, true, GUO>(I, A, B, x, y, tile_slot, corr, cmask);
        else
            sweep_node<T, M, II_LBM_SRT, false, GUO>(I, A, B, x, y, tile_slot, corr, cmask);
    } else {
        if (I.bounded)
            sweep_node<T, M, II_LBM_MRT, true, GUO>(I, A, B, x, y, tile_slot, corr, cmask);
        else
            sweep_node<T, M, II_LBM_MRT, false, GUO>(I, A, B, x, y, tile_slot, corr, cmask);
    }
}

template <typename T, typename M, bool GUO>
static hipError_t sweep_batch_g(const Batch& b, const DevPtrs& P, const void* A, void* B, int par,
                                hipStream_t s)
{
    const dim3 g(b.sweep_units);
    switch (b.sweep_unit) {
    case 128:
        hipLaunchKernelGGL((k_sweep_batch<T, M, 128, GUO>), g, dim3(128), 0, s, b.insts,
                           b.sweep_table, (const T*)A, (T*)B, P.tile_slot[par], P.corr[par],
                           P.cmask[par]);
        break;
    case 512:
        hipLaunchKernelGGL((k_sweep_batch<T, M, 512, GUO>), g, dim3(512), 0, s, b.insts,
                           b.sweep_table, (const T*)A, (T*)B, P.tile_slot[par], P.corr[par],
                           P.cmask[par]);
        break;
    default:
        hipLaunchKernelGGL((k_sweep_batch<T, M, 256, GUO>), g, dim3(256), 0, s, b.insts,
                           b.sweep_table, (const T*)A, (T*)B, P.tile_slot[par], P.corr[par],
                           P.cmask[par]);
    }
    return hipGetLastError();
}

template <typename T, typename M>
static hipError_t sweep_batch_m(const Batch& b, const DevPtrs& P, const void* A, void* B, int par,
                                hipStream_t s)
{
    return b.guo ? sweep_batch_g<T, M, true>(b, P, A, B, par, s)
                 : sweep_batch_g<T, M, false>(b, P, A, B, par, s);
}

hipError_t launch_sweep_batch(const Batch& b, const DevPtrs& P, const void* A, void* B, int par,
                              hipStream_t s)
{
    if (b.sweep_units == 0) return hipSuccess;
    if (b.storage == II_LBM_FP16)
        return b.math == II_LBM_MATH_FP64 ? sweep_batch_m<_Float16, double>(b, P, A, B, par, s)
                                          : sweep_batch_m<_Float16, float>(b, P, A, B, par, s);
    return b.math == II_LBM_MATH_FP64 ? sweep_batch_m<float, double>(b, P, A, B, par, s)
                                      : sweep_batch_m<float, float>(b, P, A, B, par, s);
}

template <typename T, typename M, int COLL, bool BOUNDED, int BX>
static hipError_t sweep_b(const InstDev& I, const DevPtrs& P, const void* A, void* B,
                          int par, hipStream_t s)
{
    const int bxn = (I.nx + BX - 1) / BX;
    if (I.guo)
        hipLaunchKernelGGL((k_sweep<T, M, COLL, BOUNDED, BX, true>), dim3(bxn * I.ny), dim3(BX), 0,
                           s, I, (const T*)A, (T*)B, bxn, P.tile_slot[par], P.corr[par],
                           P.cmask[par]);
    else
        hipLaunchKernelGGL((k_sweep<T, M, COLL, BOUNDED, BX, false>), dim3(bxn * I.ny), dim3(BX),
                           0, s, I, (const T*)A, (T*)B, bxn, P.tile_slot[par], P.corr[par],
                           P.cmask[par]);
    return hipGetLastError();
}

template <typename T, typename M, int COLL, bool BOUNDED>
static hipError_t sweep_t(const InstDev& I, const DevPtrs& P, const void* A, void* B, int par,
                          hipStream_t s)
{
    if (I.nx % 512 == 0) return sweep_b<T, M, COLL, BOUNDED, 512>(I, P, A, B, par, s);
    if (I.nx % 256 == 0) return sweep_b<T, M, COLL, BOUNDED, 256>(I, P, A, B, par, s);
    return sweep_b<T, M, COLL, BOUNDED, 64>(I, P, A, B, par, s);
}

template <typename T, typename M>
static hipError_t sweep_m(const InstDev& I, const DevPtrs& P, const void* A, void* B, int par,
                          hipStream_t s)
{
    if (I.collision == II_LBM_SRT)
        return I.bounded ? sweep_t<T, M, II_LBM_SRT, true>(I, P, A, B, par, s)
                         : sweep_t<T, M, II_LBM_SRT, false>(I, P, A, B, par, s);
    return I.bounded ? sweep_t<T, M, II_LBM_MRT, true>(I, P, A, B, par, s)
                     : sweep_t<T, M, II_LBM_MRT, false>(I, P, A, B, par, s);
}

template <typename T>
static hipError_t sweep_s(const InstDev& I, const DevPtrs& P, const void* A, void* B, int par,
                          hipStream_t s)
{
    return I.math == II_LBM_MATH_FP64 ? sweep_m<T, double>(I, P, A, B, par, s)
                                      : sweep_m<T, float>(I, P, A, B, par, s);
}

hipError_t launch_sweep(const InstDev& I, const DevPtrs& P, const void* A, void* B, int par,
                        hipStream_t s)
{
    return I.storage == II_LBM_FP16 ? sweep_s<_Float16>(I, P, A, B, par, s)
                                    : sweep_s<float>(I, P, A, B, par, s);
}

// ---------------------------------------------------------------------------
// Zero fill (rest state d = 0) of one instance's lattice region.
// ---------------------------------------------------------------------------
template <typename T>
__global__ void k_fill_zero(T* p, long long n)
{
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x)
        p[i] = (T)0;
}

hipError_t launch_fill_zero(const InstDev& I, void* A, hipStream_t s)
{
    const long long n = 9 * I.plane;
    if (I.storage == II_LBM_FP16)
        hipLaunchKernelGGL(k_fill_zero<_Float16>, dim3(2048), dim3(256), 0, s,
                           (_Float16*)A + I.lat_off, n);
    else
        hipLaunchKernelGGL(k_fill_zero<float>, dim3(2048), dim3(256), 0, s, (float*)A + I.lat_off,
                           n);
    return hipGetLastError();
}

__global__ void k_fill_ints(int* p, long long n, int value)
{
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x)
        p[i] = value;
}

hipError_t launch_fill_ints(int* p, long long n, int value, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill_ints, dim3(1024), dim3(256), 0, s, p, n, value);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Field readout of f^n: planes in bit order RHO, UX, UY, P, DISTRIB(9).
// ---------------------------------------------------------------------------
template <typename T, typename M, typename O>
__global__ void k_fields(InstDev I, const T* __restrict__ A, uint32_t what, O* __restrict__ out)
{
    const long long n = (long long)I.nx * I.ny;
    for (long long id = blockIdx.x * (long long)blockDim.x + threadIdx.x; id < n;
         id += (long long)gridDim.x * blockDim.x) {
        const int x = (int)(id % I.nx), y = (int)(id / I.nx);
        M d[9];
        gather<T, M>(I, A, x, y, d);
        double r = 0.0, ux = 0.0, uy = 0.0;
#pragma unroll
        for (int i = 0; i < 9; i++) {
            r += (double)d[i];
            ux += (double)EX[i] * (double)d[i];
            uy += (double)EY[i] * (double)d[i];
        }
        const double rho = 1.0 + r;
        long long o = 0;
        if (what & II_LBM_F_RHO) { out[o + id] = (O)rho; o += n; }
        if (what & II_LBM_F_UX) { out[o + id] = (O)ux; o += n; }
        if (what & II_LBM_F_UY) { out[o + id] = (O)uy; o += n; }
        if (what & II_LBM_F_P) { out[o + id] = (O)(rho / 3.0); o += n; }
        if (what & II_LBM_F_DISTRIB) {
#pragma unroll
            for (int i = 0; i < 9; i++) out[o + i * n + id] = (O)(WD[i] + (double)d[i]);
        }
    }
}

template <typename T, typename M>
static hipError_t fields_t(const InstDev& I, const void* A, uint32_t what, void* out, int dtype,
                           hipStream_t s)
{
    if (dtype == II_LBM_DT_F64)
        hipLaunchKernelGGL((k_fields<T, M, double>), dim3(1024), dim3(256), 0, s, I, (const T*)A,
                           what, (double*)out);
    else
        hipLaunchKernelGGL((k_fields<T, M, float>), dim3(1024), dim3(256), 0, s, I, (const T*)A,
                           what, (float*)out);
    return hipGetLastError();
}

hipError_t launch_fields(const InstDev& I, const void* A, uint32_t what, void* out, int dtype,
                         hipStream_t s)
{
    if (I.math == II_LBM_MATH_FP64)
        return I.storage == II_LBM_FP16 ? fields_t<_Float16, double>(I, A, what, out, dtype, s)
                                        : fields_t<float, double>(I, A, what, out, dtype, s);
    return I.storage == II_LBM_FP16 ? fields_t<_Float16, float>(I, A, what, out, dtype, s)
                                    : fields_t<float, float>(I, A, what, out, dtype, s);
}

// ---------------------------------------------------------------------------
// Set the stored lattice so that the next pull yields the given f (FP64,
// [9][ny][nx]): stored_i(x) = f_i(x + e_i) - w_i.
// ---------------------------------------------------------------------------
template <typename T>
__global__ void k_set_distrib(InstDev I, const double* __restrict__ f, T* __restrict__ A)
{
    const long long n = (long long)I.nx * I.ny;
    for (long long id = blockIdx.x * (long long)blockDim.x + threadIdx.x; id < n;
         id += (long long)gridDim.x * blockDim.x) {
        const int x = (int)(id % I.nx), y = (int)(id / I.nx);
#pragma unroll
        for (int i = 0; i < 9; i++) {
            int xd = x + EX[i], yd = y + EY[i];
            if (I.px) xd = (xd + I.nx) % I.nx;
            if (I.py) yd = (yd + I.ny) % I.ny;
            if (xd < 0 || xd >= I.nx || yd < 0 || yd >= I.ny) { xd = x; yd = y; }
            const double v = f[(long long)i * n + (long long)yd * I.nx + xd] - WD[i];
            Store<T>::st(A + I.lat_off + i * I.plane + (long long)y * I.pitch + x, (float)v,
                         I.inv_scale);
        }
    }
}

hipError_t launch_set_distrib(const InstDev& I, const double* f, void* A, hipStream_t s)
{
    if (I.storage == II_LBM_FP16)
        hipLaunchKernelGGL(k_set_distrib<_Float16>, dim3(1024), dim3(256), 0, s, I, f,
                           (_Float16*)A);
    else
        hipLaunchKernelGGL(k_set_distrib<float>, dim3(1024), dim3(256), 0, s, I, f, (float*)A);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// FP64 partial sums of (sum d, sum ux, sum uy, non-finite count) per block;
// the host adds the partials in block order (deterministic).
// ---------------------------------------------------------------------------
template <typename T, typename M>
__global__ __launch_bounds__(256) void k_diag(InstDev I, const T* __restrict__ A,
                                              double* __restrict__ part)
{
    __shared__ double sh[4][256];
    const long long n = (long long)I.nx * I.ny;
    double r = 0.0, ux = 0.0, uy = 0.0, bad = 0.0;
    for (long long id = blockIdx.x * (long long)blockDim.x + threadIdx.x; id < n;
         id += (long long)gridDim.x * blockDim.x) {
        const int x = (int)(id % I.nx), y = (int)(id / I.nx);
        M d[9];
        gather<T, M>(I, A, x, y, d);
#pragma unroll
        for (int i = 0; i < 9; i++) {
            if (!isfinite(d[i])) bad += 1.0;
            r += (double)d[i];
            ux += (double)EX[i] * (double)d[i];
            uy += (double)EY[i] * (double)d[i];
        }
    }
    const int t = threadIdx.x;
    sh[0][t] = r; sh[1][t] = ux; sh[2][t] = uy; sh[3][t] = bad;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (t < w)
            for (int c = 0; c < 4; c++) sh[c][t] += sh[c][t + w];
        __syncthreads();
    }
    if (t == 0)
        for (int c = 0; c < 4; c++) part[4 * blockIdx.x + c] = sh[c][0];
}

hipError_t launch_diag(const InstDev& I, const void* A, double* partials, int nblocks,
                       hipStream_t s)
{
    if (I.storage == II_LBM_FP16) {
        if (I.math == II_LBM_MATH_FP64)
            hipLaunchKernelGGL((k_diag<_Float16, double>), dim3(nblocks), dim3(256), 0, s, I,
                               (const _Float16*)A, partials);
        else
            hipLaunchKernelGGL((k_diag<_Float16, float>), dim3(nblocks), dim3(256), 0, s, I,
                               (const _Float16*)A, partials);
    } else {
        if (I.math == II_LBM_MATH_FP64)
            hipLaunchKernelGGL((k_diag<float, double>), dim3(nblocks), dim3(256), 0, s, I,
                               (const float*)A, partials);
        else
            hipLaunchKernelGGL((k_diag<float, float>), dim3(nblocks), dim3(256), 0, s, I,
                               (const float*)A, partials);
    }
    return hipGetLastError();
}

}  // namespace iilbm
