// C ABI of the learned surrogate (declared in include/gs.h): workspace
// layout, parameter handling, forward (prediction), loss and gradients
// (backpropagation through the four convolution layers) and Adam.
#include "../../include/gs.h"
#include "gs_internal.hpp"
#include "gs_launch.hpp"
#include "gs_surrogate.hpp"

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <vector>

using namespace gsapi;

namespace {

const uint32_t k_surr_magic = 0x47535347u; // "GSSG"
const int k_chan[5] = {4, 32, 32, 32, 2};  // real channels per layer boundary
const int k_cins[4] = {8, 32, 32, 32};     // stored input channels of layers 1..4
const int k_nt[4] = {2, 2, 2, 1};          // 16-wide output tiles of layers 1..4
// The input stores (u_hi, v_hi, f, k, u_lo, v_lo, 0, 0): u and v as BF16
// pairs whose low parts share the weights of the high parts.
const int k_lo_pairs = 2;

int nchunks(int cins) { return (27 * cins + 31) / 32; }

size_t a256(size_t x) { return (x + 255) / 256 * 256; }

struct Layout {
    size_t x0, z[3], a[3], pu, pv, dz[3], dz4, par, grad, m, v, wf[4], wd[4], wpart, cpart, lpart, fk, total;
};

Layout layout(size_t cells, int B)
{
    Layout L;
    size_t o = 0;
    auto take = [&](size_t bytes) {
        const size_t r = o;
        o = a256(o + bytes);
        return r;
    };
    const size_t rows = cells * (size_t)B;
    L.x0 = take(rows * 8 * 2);
    for (int i = 0; i < 3; ++i) {
        L.z[i] = take(rows * 32 * 2);
        L.a[i] = take(rows * 32 * 2);
    }
    L.pu = take(rows * 4);
    L.pv = take(rows * 4);
    // dz[l]: gradient of the loss with respect to layer l's pre-activation
    for (int i = 0; i < 3; ++i) L.dz[i] = take(rows * 32 * 2);
    L.dz4 = take(rows * 8 * 2);
    L.par = take(GS_SURR_NPARAMS * 4);
    L.grad = take(GS_SURR_NPARAMS * 4);
    L.m = take(GS_SURR_NPARAMS * 4);
    L.v = take(GS_SURR_NPARAMS * 4);
    for (int l = 0; l < 4; ++l) L.wf[l] = take((size_t)nchunks(k_cins[l]) * k_nt[l] * 512 * 2);
    // data-gradient weights of layers 2..4: input channels = the layer's stored output channels
    for (int l = 1; l < 4; ++l) L.wd[l] = take((size_t)nchunks(l == 3 ? 8 : 32) * 2 * 512 * 2);
    L.wd[0] = 0;
    L.wpart = take((size_t)gs::nn::wgrad_blocks() * 27 * 32 * 32 * 4);
    L.cpart = take((size_t)gs::nn::wgrad_blocks() * 32 * 4);
    L.lpart = take((size_t)gs::nn::loss_blocks() * 8);
    L.fk = take((size_t)B * 2 * 4);
    L.total = o;
    return L;
}

// Offsets of W_l and b_l inside the flat parameter vector (per layer: W with
// shape [c_out][c_in][27] row-major, then b[c_out]).
size_t w_off(int l)
{
    size_t o = 0;
    for (int i = 0; i < l; ++i) o += (size_t)k_chan[i + 1] * k_chan[i] * 27 + k_chan[i + 1];
    return o;
}
size_t b_off(int l) { return w_off(l) + (size_t)k_chan[l + 1] * k_chan[l] * 27; }

} // namespace

struct gs_surrogate {
    uint32_t magic;
    gs::nn::Geo geo;
    int max_batch;
    char *ws;
    Layout L;
    hipStream_t stream;
    int adam_t;
    int last_batch; // samples of the last loss_grad (gradient present when > 0)
    int last_fwd;   // samples of the last forward pass (predict or loss_grad)
    bool last_fwd_loss; // the last forward pass was loss_grad's (prediction and data gradients match it)
};

namespace {

gs_status scheck(gs_surrogate *s)
{
    if (!s || s->magic != k_surr_magic) return fail(GS_ERR_STATE, "invalid or destroyed surrogate handle");
    return GS_OK;
}

template <typename T> T *at(gs_surrogate *s, size_t off) { return reinterpret_cast<T *>(s->ws + off); }

gs_status geo_check(int32_t nx, int32_t ny, int32_t nz)
{
    if (nx < 16 || ny < 4 || nz < 4 || nx % 16 != 0)
        return fail(GS_ERR_UNSUPPORTED, "surrogate grid %dx%dx%d: need nx %% 16 == 0, nx >= 16, ny, nz >= 4", nx, ny, nz);
    if (((size_t)nx * ny * nz) % 32 != 0) return fail(GS_ERR_UNSUPPORTED, "surrogate grid cell count must be a multiple of 32");
    if ((double)nx * ny * nz > 1.0e9) return fail(GS_ERR_UNSUPPORTED, "surrogate grid too large");
    return GS_OK;
}

hipError_t repack_all(gs_surrogate *s)
{
    const float *P = at<float>(s, s->L.par);
    hipError_t e = hipSuccess;
    for (int l = 0; l < 4 && e == hipSuccess; ++l)
        e = gs::nn::launch_repack(P + w_off(l), k_chan[l + 1], k_chan[l], k_cins[l], k_nt[l], nchunks(k_cins[l]), 0,
                                  l == 0 ? k_lo_pairs : 0, at<uint16_t>(s, s->L.wf[l]), s->stream);
    for (int l = 1; l < 4 && e == hipSuccess; ++l) {
        const int cins = l == 3 ? 8 : 32;
        e = gs::nn::launch_repack(P + w_off(l), k_chan[l + 1], k_chan[l], cins, 2, nchunks(cins), 1, 0,
                                  at<uint16_t>(s, s->L.wd[l]), s->stream);
    }
    return e;
}

gs_status upload_fk(gs_surrogate *s, int32_t nsamp, const double *F, const double *k)
{
    std::vector<float> fk(2 * (size_t)nsamp);
    for (int i = 0; i < nsamp; ++i) {
        if (!std::isfinite(F[i]) || !std::isfinite(k[i])) return fail(GS_ERR_INVALID_ARG, "F/k of sample %d not finite", i);
        fk[2 * i] = (float)F[i];
        fk[2 * i + 1] = (float)k[i];
    }
    hipError_t e = hipMemcpyAsync(at<float>(s, s->L.fk), fk.data(), fk.size() * 4, hipMemcpyHostToDevice, s->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(s->stream); // fk is a stack vector
    return e == hipSuccess ? GS_OK : hip_fail(e, "F/k upload");
}

// Planes per workgroup chunk of the convolutions for a batch of nsamp
// samples: long chunks amortise the two extra ring planes (at 4 x 128^3 the
// 32 -> 32 forward takes 0.757, 0.721 and 0.699 ms with 16, 32 and 64
// planes), shorter ones keep at least 2048 workgroups (eight per CU) in flight
// on small grids and batches.
int conv_zc(const gs_surrogate *s, int nsamp)
{
    const size_t patches = (size_t)(s->geo.nx / 16) * ((s->geo.ny + 3) / 4) * (size_t)nsamp;
    int zc = 64;
    while (zc > 4 && patches * ((s->geo.nz + zc - 1) / zc) < 2048) zc /= 2;
    return zc < s->geo.nz ? zc : s->geo.nz;
}

// Forward pass of nsamp samples; keeps the activations, and the
// pre-activations too when keep_pre (the backward pass needs them; a
// prediction does not, and skips their stores).
hipError_t forward(gs_surrogate *s, int32_t nsamp, int io_f64, const void *u, const void *v, void *uo, void *vo,
                   bool keep_pre)
{
    using namespace gs::nn;
    hipError_t e = launch_pack_input(io_f64, u, v, at<float>(s, s->L.fk), nsamp, s->geo.ncell,
                                     at<uint16_t>(s, s->L.x0), s->stream);
    const float *P = at<float>(s, s->L.par);
    const uint16_t *in = at<uint16_t>(s, s->L.x0);
    for (int l = 0; l < 3 && e == hipSuccess; ++l) {
        ConvArgs a = {};
        a.geo = s->geo;
        a.nsamp = nsamp;
        a.zc = conv_zc(s, nsamp);
        a.in = in;
        a.wpack = at<uint16_t>(s, s->L.wf[l]);
        a.bias = P + b_off(l);
        a.zout = keep_pre ? at<uint16_t>(s, s->L.z[l]) : nullptr;
        a.aout = at<uint16_t>(s, s->L.a[l]);
        e = launch_conv(k_cins[l], 2, keep_pre ? MODE_HIDDEN : MODE_ACT, 0, a, s->stream);
        in = a.aout;
    }
    if (e == hipSuccess) {
        ConvArgs a = {};
        a.geo = s->geo;
        a.nsamp = nsamp;
        a.zc = conv_zc(s, nsamp);
        a.in = in;
        a.wpack = at<uint16_t>(s, s->L.wf[3]);
        a.bias = P + b_off(3);
        a.res_u = u;
        a.res_v = v;
        a.out_u = uo;
        a.out_v = vo;
        e = launch_conv(32, 1, MODE_OUT, io_f64, a, s->stream);
    }
    return e;
}

} // namespace

extern "C" {

size_t gs_surrogate_workspace_bytes(int32_t nx, int32_t ny, int32_t nz, int32_t max_batch)
{
    if (geo_check(nx, ny, nz) != GS_OK || max_batch < 1) return 0;
    return layout((size_t)nx * ny * nz, max_batch).total;
}

gs_status gs_surrogate_init(int32_t nx, int32_t ny, int32_t nz, int32_t max_batch, const float *params,
                            void *workspace, size_t workspace_bytes, void *hip_stream, gs_surrogate **out)
{
    if (!out) return fail(GS_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    gs_status st = geo_check(nx, ny, nz);
    if (st != GS_OK) return st;
    if (max_batch < 1) return fail(GS_ERR_INVALID_ARG, "max_batch < 1");
    if (!params) return fail(GS_ERR_INVALID_ARG, "params is NULL");
    for (int i = 0; i < GS_SURR_NPARAMS; ++i)
        if (!std::isfinite(params[i])) return fail(GS_ERR_INVALID_ARG, "parameter %d is not finite", i);
    const Layout L = layout((size_t)nx * ny * nz, max_batch);
    if (!workspace || !aligned(workspace, 256)) return fail(GS_ERR_INVALID_ARG, "workspace must be 256-byte aligned");
    if (workspace_bytes < L.total) return fail(GS_ERR_INVALID_ARG, "workspace holds %zu bytes, needs %zu", workspace_bytes, L.total);
    gs_surrogate *s = new (std::nothrow) gs_surrogate();
    if (!s) return fail(GS_ERR_INVALID_ARG, "out of host memory");
    s->magic = k_surr_magic;
    s->geo = gs::nn::Geo{nx, ny, nz, nx * ny * nz};
    s->max_batch = max_batch;
    s->ws = (char *)workspace;
    s->L = L;
    s->stream = (hipStream_t)hip_stream;
    s->adam_t = 0;
    s->last_batch = 0;
    s->last_fwd = 0;
    s->last_fwd_loss = false;
    st = gs_surrogate_set_params(s, params);
    if (st != GS_OK) {
        s->magic = 0;
        delete s;
        return st;
    }
    *out = s;
    return GS_OK;
}

gs_status gs_surrogate_set_params(gs_surrogate *s, const float *params)
{
    gs_status st = scheck(s);
    if (st != GS_OK) return st;
    if (!params) return fail(GS_ERR_INVALID_ARG, "params is NULL");
    hipError_t e = hipMemcpyAsync(at<float>(s, s->L.par), params, GS_SURR_NPARAMS * 4, hipMemcpyHostToDevice, s->stream);
    if (e == hipSuccess) e = hipMemsetAsync(at<float>(s, s->L.m), 0, GS_SURR_NPARAMS * 4, s->stream);
    if (e == hipSuccess) e = hipMemsetAsync(at<float>(s, s->L.v), 0, GS_SURR_NPARAMS * 4, s->stream);
    if (e == hipSuccess) e = repack_all(s);
    if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
    if (e != hipSuccess) return hip_fail(e, "surrogate parameter upload");
    s->adam_t = 0;
    s->last_batch = 0;
    return GS_OK;
}

gs_status gs_surrogate_get_params(gs_surrogate *s, float *params)
{
    gs_status st = scheck(s);
    if (st != GS_OK) return st;
    if (!params) return fail(GS_ERR_INVALID_ARG, "params is NULL");
    hipError_t e = hipMemcpyAsync(params, at<float>(s, s->L.par), GS_SURR_NPARAMS * 4, hipMemcpyDeviceToHost, s->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
    return e == hipSuccess ? GS_OK : hip_fail(e, "surrogate parameter download");
}

gs_status gs_surrogate_predict(gs_surrogate *s, int32_t nsamp, int32_t io_storage, const void *u, const void *v,
                               const double *F, const double *k, void *u_out, void *v_out)
{
    gs_status st = scheck(s);
    if (st != GS_OK) return st;
    if (nsamp < 1 || nsamp > s->max_batch) return fail(GS_ERR_INVALID_ARG, "nsamp %d outside [1, %d]", nsamp, s->max_batch);
    if (io_storage != GS_F64 && io_storage != GS_F32) return fail(GS_ERR_UNSUPPORTED, "surrogate I/O is FP64 or FP32");
    if (!u || !v || !u_out || !v_out || !F || !k) return fail(GS_ERR_INVALID_ARG, "NULL pointer");
    if (u_out == u || v_out == v || u_out == v || v_out == u) return fail(GS_ERR_INVALID_ARG, "outputs must not alias inputs");
    if ((st = upload_fk(s, nsamp, F, k)) != GS_OK) return st;
    hipError_t e = forward(s, nsamp, io_storage == GS_F64, u, v, u_out, v_out, false);
    if (e != hipSuccess) return hip_fail(e, "surrogate forward");
    s->last_fwd = nsamp;
    s->last_fwd_loss = false; // the stored data gradients no longer match the activations
    return GS_OK;
}

gs_status gs_surrogate_loss_grad(gs_surrogate *s, int32_t nsamp, const float *u, const float *v, const float *u_target,
                                 const float *v_target, const double *F, const double *k, double *loss,
                                 float *grad_host)
{
    using namespace gs::nn;
    gs_status st = scheck(s);
    if (st != GS_OK) return st;
    if (nsamp < 1 || nsamp > s->max_batch) return fail(GS_ERR_INVALID_ARG, "nsamp %d outside [1, %d]", nsamp, s->max_batch);
    if (!u || !v || !u_target || !v_target || !F || !k) return fail(GS_ERR_INVALID_ARG, "NULL pointer");
    if ((st = upload_fk(s, nsamp, F, k)) != GS_OK) return st;
    const size_t rows = (size_t)nsamp * s->geo.ncell;
    float *pu = at<float>(s, s->L.pu), *pv = at<float>(s, s->L.pv);
    hipError_t e = forward(s, nsamp, 0, u, v, pu, pv, true);
    const double n_terms = 2.0 * (double)rows;
    uint16_t *dz4 = at<uint16_t>(s, s->L.dz4);
    if (e == hipSuccess)
        e = launch_loss_grad(pu, pv, u_target, v_target, rows, (float)(2.0 / n_terms), dz4, at<double>(s, s->L.lpart),
                             s->stream);
    float *G = at<float>(s, s->L.grad);
    float *wpart = at<float>(s, s->L.wpart), *cpart = at<float>(s, s->L.cpart);
    // layer l (0-based) consumes act_in[l]; its output gradient dz; dgrad writes into the other buffer.
    const uint16_t *act_in[4] = {at<uint16_t>(s, s->L.x0), at<uint16_t>(s, s->L.a[0]), at<uint16_t>(s, s->L.a[1]),
                                 at<uint16_t>(s, s->L.a[2])};
    const uint16_t *dz = dz4;
    int couts = 8;
    for (int l = 3; l >= 0 && e == hipSuccess; --l) {
        WgradArgs w = {};
        w.geo = s->geo;
        w.nsamp = nsamp;
        w.dz = dz;
        w.act = act_in[l];
        w.part = wpart;
        w.bpart = cpart;
        e = launch_wgrad(k_cins[l], couts, w, s->stream);
        if (e == hipSuccess)
            e = launch_wgrad_reduce(wpart, couts == 8 ? 16 : 32, k_cins[l] == 8 ? 16 : 32, k_chan[l + 1], k_chan[l],
                                    l == 0 ? k_lo_pairs : 0, G + w_off(l), s->stream);
        if (e == hipSuccess) e = launch_bias_reduce(cpart, k_chan[l + 1], G + b_off(l), s->stream);
        if (l == 0 || e != hipSuccess) break;
        ConvArgs a = {};
        a.geo = s->geo;
        a.nsamp = nsamp;
        a.zc = conv_zc(s, nsamp);
        a.in = dz;
        a.wpack = at<uint16_t>(s, s->L.wd[l]);
        a.zprev = at<uint16_t>(s, s->L.z[l - 1]);
        a.aout = at<uint16_t>(s, s->L.dz[l - 1]);
        e = launch_conv(couts, 2, MODE_DGRAD, 0, a, s->stream);
        dz = a.aout;
        couts = 32;
    }
    std::vector<double> lp(loss_blocks());
    if (e == hipSuccess)
        e = hipMemcpyAsync(lp.data(), at<double>(s, s->L.lpart), lp.size() * 8, hipMemcpyDeviceToHost, s->stream);
    if (e == hipSuccess && grad_host)
        e = hipMemcpyAsync(grad_host, G, GS_SURR_NPARAMS * 4, hipMemcpyDeviceToHost, s->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
    if (e != hipSuccess) return hip_fail(e, "surrogate backward");
    double sum = 0.0;
    for (double x : lp) sum += x;
    if (loss) *loss = sum / n_terms;
    s->last_batch = nsamp;
    s->last_fwd = nsamp;
    s->last_fwd_loss = true;
    return GS_OK;
}

gs_status gs_surrogate_adam(gs_surrogate *s, float lr, float beta1, float beta2, float eps)
{
    gs_status st = scheck(s);
    if (st != GS_OK) return st;
    if (s->last_batch == 0) return fail(GS_ERR_STATE, "no gradient: call gs_surrogate_loss_grad first");
    if (!(lr > 0) || !(beta1 >= 0 && beta1 < 1) || !(beta2 >= 0 && beta2 < 1) || !(eps > 0))
        return fail(GS_ERR_INVALID_ARG, "bad Adam hyper-parameters");
    s->adam_t += 1;
    const float c1 = 1.f - std::pow(beta1, (float)s->adam_t), c2 = 1.f - std::pow(beta2, (float)s->adam_t);
    hipError_t e = gs::nn::launch_adam(at<float>(s, s->L.par), at<float>(s, s->L.grad), at<float>(s, s->L.m),
                                       at<float>(s, s->L.v), GS_SURR_NPARAMS, lr, beta1, beta2, eps, c1, c2, s->stream);
    if (e == hipSuccess) e = repack_all(s);
    return e == hipSuccess ? GS_OK : hip_fail(e, "Adam step");
}

gs_status gs_surrogate_read_tensor(gs_surrogate *s, int32_t tensor, int32_t layer, void *host, size_t host_bytes)
{
    gs_status st = scheck(s);
    if (st != GS_OK) return st;
    if (!host) return fail(GS_ERR_INVALID_ARG, "host is NULL");
    const size_t rows = (size_t)s->last_fwd * s->geo.ncell;
    size_t off = 0, bytes = 0;
    switch (tensor) {
    case GS_SURR_INPUT:
        if (layer != 0) return fail(GS_ERR_INVALID_ARG, "the input has layer 0 only");
        off = s->L.x0, bytes = rows * 8 * 2;
        break;
    case GS_SURR_PRE:
    case GS_SURR_ACT:
        if (layer < 0 || layer > 2) return fail(GS_ERR_INVALID_ARG, "hidden layer %d outside [0, 2]", layer);
        if (tensor == GS_SURR_PRE && s->last_fwd && !s->last_fwd_loss)
            return fail(GS_ERR_STATE, "a prediction keeps no pre-activations: call gs_surrogate_loss_grad first");
        off = tensor == GS_SURR_PRE ? s->L.z[layer] : s->L.a[layer], bytes = rows * 32 * 2;
        break;
    case GS_SURR_PRED:
        if (layer != 3) return fail(GS_ERR_INVALID_ARG, "the prediction is layer 3's");
        if (!s->last_fwd_loss) return fail(GS_ERR_STATE, "no prediction kept: call gs_surrogate_loss_grad first");
        off = s->L.pu, bytes = rows * 4;
        break;
    case GS_SURR_DOUT:
        if (layer != 3) return fail(GS_ERR_INVALID_ARG, "the output gradient is layer 3's");
        off = s->L.dz4, bytes = rows * 8 * 2;
        break;
    case GS_SURR_DPRE:
        if (layer < 0 || layer > 2) return fail(GS_ERR_INVALID_ARG, "hidden layer %d outside [0, 2]", layer);
        off = s->L.dz[layer], bytes = rows * 32 * 2;
        break;
    default:
        return fail(GS_ERR_INVALID_ARG, "unknown tensor %d", tensor);
    }
    if ((tensor == GS_SURR_DOUT || tensor == GS_SURR_DPRE) && !s->last_fwd_loss)
        return fail(GS_ERR_STATE, "no backward pass since the last forward pass");
    if (rows == 0) return fail(GS_ERR_STATE, "no forward pass yet");
    if (tensor == GS_SURR_PRED) {
        if (host_bytes < 2 * bytes) return fail(GS_ERR_INVALID_ARG, "host holds %zu bytes, needs %zu", host_bytes, 2 * bytes);
    } else if (host_bytes < bytes) {
        return fail(GS_ERR_INVALID_ARG, "host holds %zu bytes, needs %zu", host_bytes, bytes);
    }
    hipError_t e = hipMemcpyAsync(host, s->ws + off, bytes, hipMemcpyDeviceToHost, s->stream);
    if (e == hipSuccess && tensor == GS_SURR_PRED)
        e = hipMemcpyAsync((char *)host + bytes, s->ws + s->L.pv, bytes, hipMemcpyDeviceToHost, s->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
    return e == hipSuccess ? GS_OK : hip_fail(e, "surrogate tensor read");
}

gs_status gs_surrogate_destroy(gs_surrogate *s)
{
    gs_status st = scheck(s);
    if (st != GS_OK) return st;
    hipError_t e = hipStreamSynchronize(s->stream);
    s->magic = 0;
    delete s;
    return e == hipSuccess ? GS_OK : hip_fail(e, "surrogate destroy sync");
}

} // extern "C"
