// sc_unet.h -- host objects of the denoiser network.
#pragma once
#include <stdint.h>

#include <vector>

#include "sc_internal.h"

namespace scl {

constexpr uint32_t kUnetIn = 9;    // log1p(rgb) x3, albedo, normal x3, depth/10, transparent
constexpr uint32_t kUnetOut = 3;   // predicted log1p(rgb)

struct UnetLayer {
    uint32_t cout, ks, cin;
    uint32_t cout_p, cin_p, kpad, kpad_t;
    size_t w_off, b_off;    // into the float parameter vector
    size_t wf_off, wd_off;  // into the bf16 forward / input-gradient matrices
};

// element offsets (bf16 units) of the activation and gradient tensors
struct UnetTensors {
    size_t in = 0, g0 = 0, g2 = 0;
    std::vector<size_t> pool, pool_idx, enc_a, enc_b, cat, dec_a, dec_b, skip;
    void clear() {
        pool.clear(); pool_idx.clear(); enc_a.clear(); enc_b.clear();
        cat.clear(); dec_a.clear(); dec_b.clear(); skip.clear();
    }
};

struct Unet {
    Ctx* ctx = nullptr;
    std::vector<uint32_t> widths;
    std::vector<UnetLayer> layers;
    size_t n_params = 0;
    DevBuf theta, m, v, grad, wf, wd, loss, acts, pred;
    uint32_t B = 0, H = 0, W = 0;
    UnetTensors t;
    uint64_t step = 0;
    bool cat_valid = false;   // the last forward pass kept what a backward pass reads
    bool grad_clear = false;  // grad holds zeros (the Adam step clears it as it reads it)
    uint32_t cus = 256;       // compute units of the device (sizes the persistent convolution grid)
};

sc_status unet_create(Ctx* c, const uint32_t* widths, uint32_t levels, Unet* u);
sc_status unet_refresh(Unet* u);
sc_status unet_prepare(Unet* u, uint32_t B, uint32_t H, uint32_t W);
sc_status unet_pack_input(Unet* u, const float* feat);
sc_status unet_pack_dpred(Unet* u, const float* dpred);
// keep_cat: materialise the decoder concatenations (needed by a backward
// pass); inference reads them in place.
sc_status unet_forward_packed(Unet* u, bool keep_cat = true);
sc_status unet_backward_packed(Unet* u);
sc_status unet_loss(Unet* u, const float* target, float* loss_dev);
sc_status unet_adam(Unet* u, float lr);
sc_status unet_features(Unet* u, const sc_aov& in, uint32_t w, uint32_t h);
sc_status unet_output_rgb(Unet* u, uint32_t w, uint32_t h, float* out);
// one convolution layer alone: forward (bf16 output of a 3x3 layer as
// float, float output of the 1x1 layer) and gradients (dX as float of the
// bf16 values, dW float: weights then bias); both synchronise
sc_status unet_layer_forward(Unet* u, uint32_t layer, const float* X, uint32_t n, uint32_t h, uint32_t w, int relu,
                             float* Y);
sc_status unet_layer_backward(Unet* u, uint32_t layer, const float* X, const float* dZ, uint32_t n, uint32_t h,
                              uint32_t w, float* dX, float* dW);
// the network's input features of a w x h render as float [h][w][9]
sc_status features_f32(Ctx* c, const sc_aov& in, uint32_t w, uint32_t h, float* out);

}  // namespace scl
