/*
 * ii_learned.h — learned near-interface correction of a 2x-coarsened
 * II-LBM membrane run (BF16 MFMA training and inference, FP32 accumulation).
 *
 * The paper fixes none of this part; the network and its use are:
 *  - a 16 x 16 tile of coarse nodes is corrected from a 24 x 24 input patch
 *    (4 nodes of periodic halo) through four valid 3 x 3 convolutions,
 *    channels 4 -> 32 -> 32 -> 32 -> 9, ReLU after the first three;
 *  - input channels per node: (rho - 1, u_x, u_y) of the pulled distributions
 *    (u = sum_i e_i f_i as in the method, Sec. 2.2.1) and the signed distance
 *    to the marker polygon (positive outside, clipped to [-8, 8]), each times
 *    a per-channel input scale; the three flow channels are then divided by
 *    the patch amplitude s = max(rms over the patch of their vector, 1e-6);
 *  - output: nine population corrections df_i (times the output scale and
 *    s) added
 *    to the pre-collision f_i at nodes with |sd| <= 4, except on links whose
 *    two end nodes lie on different sides of the polygon;
 *  - training target: f^eq(rho_c, u_hat) - f^eq(rho_c, u_c) (He-Luo
 *    equilibrium, Sec. 2.2.1): the change of the equilibrium that gives the
 *    coarse node the fine run's velocity u_hat = 2 u_f at fine node (2x, 2y)
 *    (diffusive scaling) at unchanged density.
 *
 * Parameters are one FP32 array of II_CNN_NPARAM values in the order
 * W1 b1 W2 b2 W3 b3 W4 b4, each W[dy][dx][ci][co] row-major.  Kernels read
 * BF16 copies packed by ii_cnn_pack into MFMA fragment order.
 *
 * All pointers are device pointers owned by the caller unless stated
 * otherwise; `stream` is a hipStream_t (NULL = default).  Calls enqueue work
 * and return without waiting; errors are II_LBM_* codes from ii_lbm.h.
 * Patch tensors: input [n][24][24][4] BF16 (as uint16), flags [n][24][24]
 * uint8 (bit 0: inside the polygon, bit 1: |sd| <= 4), output / target
 * [n][16][16][9] FP32 (network units, i.e. before the output scale and the
 * patch amplitude), mask [n][16][16] uint8, patch amplitudes pscale[n] FP32.
 */
#ifndef II_LEARNED_H
#define II_LEARNED_H

#include <stddef.h>
#include <stdint.h>

#include "ii_lbm.h"

#ifdef __cplusplus
extern "C" {
#endif

#define II_CNN_NPARAM 22281
#define II_CNN_PATCH 24
#define II_CNN_TILE 16

/* Scales between physical channels and network units. */
typedef struct ii_cnn_scales {
    float in_scale[4];   /* rho - 1, u_x, u_y, sd */
    float out_scale;     /* df_i = out_scale * network output */
} ii_cnn_scales;

/* Bytes of the packed BF16 fragment buffer. */
size_t ii_cnn_packed_bytes(void);

/* Packs the FP32 parameters into forward and backward-data fragments. */
int ii_cnn_pack(const float* params, void* packed, void* stream);

/* Forward pass over n patches: out[n][16][16][9] FP32.  When save is not
 * NULL it receives the activations of layers 1-3 (BF16, ii_cnn_save_bytes
 * per patch) for ii_cnn_backward. */
size_t ii_cnn_save_bytes(void);
int ii_cnn_forward(const float* params, const void* packed, const uint16_t* in, int32_t n,
                   float* out, uint16_t* save, void* stream);

/* Backward pass of the masked mean squared error
 *   loss = sum_{p, i} mask (out - target)^2 / (9 sum mask)
 * over the n patches (out and save from ii_cnn_forward).  Writes the
 * gradient grad[II_CNN_NPARAM] (summed over patches in a fixed order) and
 * loss[0].  `work` is scratch of ii_cnn_work_bytes(n) bytes. */
size_t ii_cnn_work_bytes(int32_t n);
int ii_cnn_backward(const float* params, const void* packed, const uint16_t* in,
                    const uint16_t* save, const float* out, const float* target,
                    const uint8_t* mask, int32_t n, float* grad, float* loss, void* work,
                    void* stream);

/* One Adam step (b1 = 0.9, b2 = 0.999, eps = 1e-8, bias-corrected, t >= 1)
 * on the FP32 parameters with moments m, v; re-packs `packed`. */
int ii_cnn_adam(float* params, const float* grad, float* m, float* v, int32_t t, float lr,
                void* packed, void* stream);

/* Band tiles of every instance of a handle at its current state: tiles
 * (16 x 16 nodes) that a chord passes within 4 + 1/2 lu of (every tile with
 * a node at |sd| <= 4 is among them).  tiles[inst * cap + r] = (tx, ty) for
 * r < count[inst], in row-major tile order (tiles holds 2 * n_inst * cap
 * int32); cap >= tiles per instance.
 * Instances must be periodic membranes whose sides are multiples of 16, with at
 * most 1024 tiles (EINVAL otherwise).  A patch near more chords than its
 * lists hold (256 within 8 lu, 16 crossings of one row) marks the instance,
 * which the next synchronising call reports as II_LBM_ECAPACITY. */
int ii_lbm_learned_tiles(ii_lbm_handle* h, int32_t cap, int32_t* tiles, int32_t* count);

/* Input patches and flags of the listed band tiles (slots inst * cap + r,
 * r < count[inst]; other slots are left alone) at the handle's current
 * state. */
int ii_lbm_learned_patches(ii_lbm_handle* h, const ii_cnn_scales* sc, int32_t cap,
                           const int32_t* tiles, const int32_t* count, uint16_t* in,
                           uint8_t* flags, float* pscale);

/* Training targets of the listed tiles, coarse handle hc against fine
 * handle hf (same instance count, fine sides twice the coarse ones), in
 * network units, and the band mask taken from flags. */
int ii_lbm_learned_targets(ii_lbm_handle* hc, ii_lbm_handle* hf, const ii_cnn_scales* sc,
                           int32_t cap, const int32_t* tiles, const int32_t* count,
                           const uint8_t* flags, const float* pscale, float* target,
                           uint8_t* mask);

/* The masked add of given corrections out[n][16][16][9] (network units) to
 * the listed tiles of the handle's current state, with the band and side
 * flags of ii_lbm_learned_patches (used, for instance, to apply the exact
 * targets of a fine run as the ideal correction). */
int ii_lbm_learned_apply(ii_lbm_handle* h, const ii_cnn_scales* sc, int32_t cap,
                         const int32_t* tiles, const int32_t* count, const uint8_t* flags,
                         const float* pscale, const float* out);

/* The network and the masked add of ii_lbm_learned_apply, fused per tile,
 * on patches from ii_lbm_learned_patches of the same state (every patch
 * must be built before any tile is corrected: a tile's halo overlaps its
 * neighbours' nodes).  Tiles with no band node are skipped.  At most 4096
 * instances per handle (EINVAL otherwise). */
int ii_lbm_learned_infer(ii_lbm_handle* h, const float* params, const void* packed,
                         const ii_cnn_scales* sc, int32_t cap, const int32_t* tiles,
                         const int32_t* count, const uint16_t* in, const uint8_t* flags,
                         const float* pscale);

/* The correction of one coarse step, in place on the handle's current
 * state: ii_lbm_learned_tiles, ii_lbm_learned_patches of the uncorrected
 * state, then ii_lbm_learned_infer.  tiles / count / in / flags are scratch of
 * the shapes above (n_inst * cap slots). */
int ii_lbm_learned_correct(ii_lbm_handle* h, const float* params, const void* packed,
                           const ii_cnn_scales* sc, int32_t cap, int32_t* tiles, int32_t* count,
                           uint16_t* in, uint8_t* flags, float* pscale);

/* Registers the correction of ii_lbm_learned_correct to be applied by the
 * handle at the end of every step (ii_lbm_step), so that the state after n
 * steps is that of n rounds of ii_lbm_step(h, 1) followed by
 * ii_lbm_learned_correct with the same arguments.  Inside a step:
 *  - band tiles and patch geometry need only the moved markers and run on
 *    an internal stream beside the sweep and the interface pass;
 *  - patch flow and the network + masked add follow the sweep on the
 *    handle's stream, beside the interface pass of the next step (which
 *    does not read the lattice).
 * Steps replayed as HIP graphs include the correction.  params, packed and
 * the scratch buffers (as for ii_lbm_learned_correct) must stay valid while
 * registered; *sc is copied.  params == NULL unregisters.  EINVAL as for
 * ii_lbm_learned_infer. */
int ii_lbm_set_learned(ii_lbm_handle* h, const float* params, const void* packed,
                       const ii_cnn_scales* sc, int32_t cap, int32_t* tiles, int32_t* count,
                       uint16_t* in, uint8_t* flags, float* pscale);

#ifdef __cplusplus
}
#endif
#endif
