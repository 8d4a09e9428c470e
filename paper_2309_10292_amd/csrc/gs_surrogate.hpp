// Internal interface of the surrogate network kernels (gs_surrogate.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace gs {
namespace nn {

// Input normalisation of the (F, k) channels.
constexpr float F_CENTER = 0.035f, F_SCALE = 0.025f;
constexpr float K_CENTER = 0.055f, K_SCALE = 0.015f;

enum { MODE_HIDDEN = 0, MODE_OUT = 1, MODE_DGRAD = 2, MODE_ACT = 3 };

struct Geo {
    int nx, ny, nz;
    int ncell; // nx * ny * nz
};

struct ConvArgs {
    Geo geo;
    int nsamp;
    int zc;                 // planes per workgroup chunk (the 32 -> 32 hidden and data-gradient kernels pick their own)
    const uint16_t *in;     // channels-last BF16 input (CIN channels)
    const uint16_t *wpack;  // packed BF16 weights (B fragments)
    const float *bias;      // MODE_HIDDEN / MODE_ACT / MODE_OUT
    uint16_t *zout;         // MODE_HIDDEN: pre-activation (32 channels)
    uint16_t *aout;         // MODE_HIDDEN / MODE_ACT: activation; MODE_DGRAD: gradient (32 channels)
    const uint16_t *zprev;  // MODE_DGRAD: pre-activation of the layer below
    const void *res_u, *res_v; // MODE_OUT: residual input (planar, sample-major)
    void *out_u, *out_v;       // MODE_OUT: prediction (planar)
};

struct WgradArgs {
    Geo geo;
    int nsamp;
    const uint16_t *dz;  // output gradient, COUTS channels
    const uint16_t *act; // layer input, CIN channels
    float *part;         // wgrad_blocks() x 27 x (16 MT) x (16 NT) partial sums
    float *bpart;        // wgrad_blocks() x 32 partial sums of dz (bias gradient)
};

hipError_t launch_conv(int cin, int nt, int mode, int io_f64, const ConvArgs &a, hipStream_t st);
int wgrad_blocks();
hipError_t launch_wgrad(int cin, int couts, const WgradArgs &a, hipStream_t st);
hipError_t launch_wgrad_reduce(const float *part, int pco, int pci, int cout, int cin, int lo_pairs, float *gW,
                               hipStream_t st);
hipError_t launch_bias_reduce(const float *bpart, int cout, float *gb, hipStream_t st);
hipError_t launch_pack_input(int io_f64, const void *u, const void *v, const float *fk, int nsamp, int ncell,
                             uint16_t *x, hipStream_t st);
int loss_blocks();
hipError_t launch_loss_grad(const float *pu, const float *pv, const float *tu, const float *tv, size_t rows,
                            float scale, uint16_t *dz4, double *part, hipStream_t st);
hipError_t launch_adam(float *p, const float *g, float *m, float *v, int n, float lr, float b1, float b2, float eps,
                       float c1, float c2, hipStream_t st);
hipError_t launch_repack(const float *W, int cout, int cin, int cins, int nt, int nch, int dgrad, int lo_pairs,
                         uint16_t *out, hipStream_t st);

} // namespace nn
} // namespace gs
