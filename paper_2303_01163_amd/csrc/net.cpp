// C ABI of the learned correction network (include/asdsm_learn.h): parameter layout, workspace,
// forward, backward and Adam, all enqueued on the network's stream.
#include <atomic>
#include <cmath>
#include <cstring>
#include <new>
#include <string>

#include "../../include/asdsm_learn.h"
#include "asdsm_internal.hpp"
#include "kernels.hpp"
#include "learn_internal.hpp"

namespace asdsm {
namespace {

#define NET_HIP_CHECK(expr)                                                                       \
    do {                                                                                          \
        hipError_t _e = (expr);                                                                   \
        if (_e != hipSuccess) return fail(ASDSM_E_DEVICE, std::string(#expr) + ": " + hipGetErrorString(_e)); \
    } while (0)

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// Deterministic normal deviates for the initial weights: splitmix64 outputs through Box-Muller.
struct InitRng {
    uint64_t s;
    uint64_t next() {
        s += 0x9E3779B97F4A7C15ull;
        uint64_t z = s;
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
        return z ^ (z >> 31);
    }
    double uniform() { return ((next() >> 11) + 0.5) * (1.0 / 9007199254740992.0); }
    double normal() {
        const double u1 = uniform(), u2 = uniform();
        return std::sqrt(-2.0 * std::log(u1)) * std::cos(6.283185307179586 * u2);
    }
};

void layout(Net &net, char *base) {
    size_t off = 0;
    auto take = [&](size_t bytes) -> char * {
        char *p = base ? base + off : nullptr;
        off = align256(off + bytes);
        return p;
    };
    const size_t np = net.nparam, nv = (size_t)net.nvox;
    net.P = (float *)take(np * 4);
    net.G = (float *)take(np * 4);
    net.M = (float *)take(np * 4);
    net.V = (float *)take(np * 4);
    size_t wmax = 0;
    for (int l = 0; l < kNetLayers; ++l) {
        const size_t nw = (size_t)kNetCoutP[l] * 27 * kNetCinP[l];
        net.Wb[l] = (unsigned short *)take(nw * 2);
        wmax = nw > wmax ? nw : wmax;
    }
    net.Wt = (unsigned short *)take(wmax * 2);
    net.act[0] = (float *)take(nv * 16 * 4);
    for (int l = 1; l < kNetLayers; ++l) net.act[l] = (float *)take(nv * 32 * 4);
    net.act[kNetLayers] = (float *)take(nv * 4);
    net.gA = (float *)take(nv * 32 * 4);
    net.gB = (float *)take(nv * 32 * 4);
    net.d16 = (float *)take(nv * 16 * 4);
    net.rho = (float *)take(nv * 4);
    net.target = nullptr;
    const size_t nblk = net_reduce_blocks(net.n);
    net.partial = (float *)take(nblk * (wmax + 64) * 4);  // per block: weights and biases of every slice
    net.nblk_loss = (int)((nv + 255) / 256);
    net.lpart = (double *)take((size_t)net.nblk_loss * 8);
    net.skip = (int *)take(2 * sizeof(int));
    net.ws_need = off;
}

int refresh_bf16(Net &net) {
    for (int l = 0; l < kNetLayers; ++l)
        net_to_bf16(net.P + net.wofs[l], net.Wb[l], kNetCoutP[l] * 27 * kNetCinP[l], net.stream);
    NET_HIP_CHECK(hipGetLastError());
    return ASDSM_OK;
}

int require_ws(const Net &net) {
    if (!net.ws) return fail(ASDSM_E_WORKSPACE, "no workspace attached (asdsm_net_set_workspace)");
    return ASDSM_OK;
}

int forward(Net &net, const float *in) {
    NET_HIP_CHECK(hipMemcpyAsync(net.act[0], in, (size_t)net.nvox * 16 * 4, hipMemcpyDeviceToDevice, net.stream));
    for (int l = 0; l < kNetLayers; ++l) {
        const bool last = (l == kNetLayers - 1);
        net_conv_fwd(net.n, kNetCinP[l], kNetCout[l], last ? 1 : 32, !last, net.act[l], l > 0, net.Wb[l],
                     net.P + net.bofs[l], net.act[l + 1], !last, nullptr, net.stream);
    }
    NET_HIP_CHECK(hipGetLastError());
    return ASDSM_OK;
}

// Backward pass from d16 (gradient of the loss with respect to the output, channel 0 of 16).
int backward(Net &net) {
    const float *g = net.d16;
    int cop_g = 16;
    float *bufs[2] = {net.gA, net.gB};
    for (int l = kNetLayers - 1; l >= 0; --l) {
        // weights and biases of layer l (contiguous in the parameter vector)
        net_conv_wgrad(net.n, kNetCinP[l], kNetCoutP[l], g, cop_g, net.act[l], l > 0, net.partial,
                       net.G + net.wofs[l], net.stream);
        if (l == 0) break;
        // data gradient: transposed, flipped weights; then the ReLU of layer l-1's output
        net_flip(net.P + net.wofs[l], kNetCoutP[l], kNetCinP[l], net.Wt, net.stream);
        float *dx = bufs[l % 2];
        net_conv_fwd(net.n, kNetCoutP[l], kNetCinP[l], kNetCinP[l], false, g, false, net.Wt, nullptr, dx, false,
                     nullptr, net.stream);
        net_relu_mask(net.nvox, kNetCinP[l], kNetCout[l - 1], reinterpret_cast<const unsigned short *>(net.act[l]),
                      dx, net.stream);
        g = dx;
        cop_g = kNetCinP[l];
    }
    NET_HIP_CHECK(hipGetLastError());
    return ASDSM_OK;
}

}  // namespace
}  // namespace asdsm

using namespace asdsm;

extern "C" {

int asdsm_net_create(asdsm_net_t *out, int n, uint64_t seed, void *hip_stream) {
    if (!out) return fail(ASDSM_E_ARG, "out must be non-NULL");
    *out = nullptr;
    if (n < 4 || n > 256) return fail(ASDSM_E_ARG, "n must be in 4..256");
    asdsm_net_s *h = new (std::nothrow) asdsm_net_s();
    if (!h) return fail(ASDSM_E_ARG, "out of host memory");
    Net &net = h->net;
    static std::atomic<uint64_t> serials{0};
    net.serial = ++serials;
    net.n = n;
    net.nvox = (long long)n * n * n;
    net.stream = (hipStream_t)hip_stream;
    size_t off = 0;
    for (int l = 0; l < kNetLayers; ++l) {
        net.wofs[l] = off;
        off += (size_t)kNetCoutP[l] * 27 * kNetCinP[l];
        net.bofs[l] = off;
        off += (size_t)kNetCoutP[l];
    }
    net.nparam = off;
    net.host_params.assign(off, 0.0f);
    // He-normal weights over the real fan-in for the hidden layers; the output layer starts at zero,
    // so that the first proposals are c = 0 and training starts from the plain residual
    InitRng rng{seed};
    for (int l = 0; l < kNetLayers; ++l) {
        const int cin_real = (l == 0) ? kNetInputChannels : kNetCout[l - 1];
        const double sd = (l == kNetLayers - 1) ? 0.0 : std::sqrt(2.0 / (27.0 * cin_real));
        for (int co = 0; co < kNetCoutP[l]; ++co)
            for (int tap = 0; tap < 27; ++tap)
                for (int ci = 0; ci < kNetCinP[l]; ++ci) {
                    const double v = rng.normal() * sd;
                    const bool real = co < kNetCout[l] && ci < cin_real;
                    net.host_params[net.wofs[l] + ((size_t)co * 27 + tap) * kNetCinP[l] + ci] = real ? (float)v : 0.f;
                }
    }
    layout(net, nullptr);
    *out = h;
    set_error("");
    return ASDSM_OK;
}

int asdsm_net_param_count(asdsm_net_t h, size_t *count) {
    if (!h || !count) return fail(ASDSM_E_ARG, "net and count must be non-NULL");
    *count = h->net.nparam;
    return ASDSM_OK;
}

int asdsm_net_workspace_size(asdsm_net_t h, size_t *bytes) {
    if (!h || !bytes) return fail(ASDSM_E_ARG, "net and bytes must be non-NULL");
    *bytes = h->net.ws_need;
    return ASDSM_OK;
}

int asdsm_net_set_workspace(asdsm_net_t h, void *dev, size_t bytes) {
    if (!h) return fail(ASDSM_E_ARG, "net must be non-NULL");
    Net &net = h->net;
    if (!dev) return fail(ASDSM_E_WORKSPACE, "workspace pointer is NULL");
    if (((uintptr_t)dev & 255u) != 0) return fail(ASDSM_E_WORKSPACE, "workspace must be 256-byte aligned");
    if (bytes < net.ws_need) return fail(ASDSM_E_WORKSPACE, "workspace too small: need " + std::to_string(net.ws_need) + " bytes");
    net.ws = dev;
    layout(net, (char *)dev);
    net_conv_prepare();  // on the current device
    if (!net.hloss) NET_HIP_CHECK(hipHostMalloc((void **)&net.hloss, (size_t)net.nblk_loss * 8, hipHostMallocDefault));
    return asdsm_net_params(h, net.host_params.data(), 0);
}

int asdsm_net_params(asdsm_net_t h, float *host, int get) {
    if (!h || !host) return fail(ASDSM_E_ARG, "net and host must be non-NULL");
    Net &net = h->net;
    if (int rc = require_ws(net)) return rc;
    const size_t bytes = net.nparam * 4;
    if (get) {
        NET_HIP_CHECK(hipMemcpyAsync(host, net.P, bytes, hipMemcpyDeviceToHost, net.stream));
    } else {
        if (host != net.host_params.data()) std::memcpy(net.host_params.data(), host, bytes);
        NET_HIP_CHECK(hipMemcpyAsync(net.P, net.host_params.data(), bytes, hipMemcpyHostToDevice, net.stream));
        NET_HIP_CHECK(hipMemsetAsync(net.M, 0, bytes, net.stream));
        NET_HIP_CHECK(hipMemsetAsync(net.V, 0, bytes, net.stream));
        net.adam_t = 0;
        if (int rc = refresh_bf16(net)) return rc;
    }
    NET_HIP_CHECK(hipStreamSynchronize(net.stream));
    set_error("");
    return ASDSM_OK;
}

int asdsm_net_forward(asdsm_net_t h, const float *in, float *out) {
    if (!h || !in || !out) return fail(ASDSM_E_ARG, "net, in and out must be non-NULL");
    Net &net = h->net;
    if (int rc = require_ws(net)) return rc;
    if (int rc = forward(net, in)) return rc;
    NET_HIP_CHECK(hipMemcpyAsync(out, net.act[kNetLayers], (size_t)net.nvox * 4, hipMemcpyDeviceToDevice, net.stream));
    set_error("");
    return ASDSM_OK;
}

int asdsm_net_gradient(asdsm_net_t h, const float *in, const float *target, int loss_kind, double *loss,
                       float *grad_host) {
    if (!h || !in || !target) return fail(ASDSM_E_ARG, "net, in and target must be non-NULL");
    Net &net = h->net;
    if (int rc = require_ws(net)) return rc;
    NetStencil K = {}, KT = {};
    if (loss_kind == ASDSM_NET_LOSS_MSE) {
        K.c[0] = KT.c[0] = 1.f;
    } else if (loss_kind == ASDSM_NET_LOSS_RESIDUAL) {
        if (!net.plan) return fail(ASDSM_E_ARG, "the residual loss needs a network bound to a plan");
        K = net.K;
        KT = net.KT;
    } else {
        return fail(ASDSM_E_ARG, "unknown loss kind");
    }
    if (int rc = forward(net, in)) return rc;
    net_stencil_loss(net.n, net.act[kNetLayers], target, K, KT, net.rho, net.d16, net.lpart, net.stream);
    if (int rc = backward(net)) return rc;
    if (!loss && !grad_host) {  // nothing to hand back: return once enqueued
        NET_HIP_CHECK(hipGetLastError());
        set_error("");
        return ASDSM_OK;
    }
    NET_HIP_CHECK(hipMemcpyAsync(net.hloss, net.lpart, (size_t)net.nblk_loss * 8, hipMemcpyDeviceToHost, net.stream));
    if (grad_host) NET_HIP_CHECK(hipMemcpyAsync(grad_host, net.G, net.nparam * 4, hipMemcpyDeviceToHost, net.stream));
    NET_HIP_CHECK(hipStreamSynchronize(net.stream));
    if (loss) {
        double s = 0.0;
        for (int b = 0; b < net.nblk_loss; ++b) s += net.hloss[b];
        *loss = s / (double)net.nvox;
    }
    set_error("");
    return ASDSM_OK;
}

int asdsm_net_bind(asdsm_net_t h, asdsm_plan_t plan) {
    if (!h || !plan) return fail(ASDSM_E_ARG, "net and plan must be non-NULL");
    Net &net = h->net;
    const Plan &p = plan->p;
    if (p.d != 3) return fail(ASDSM_E_ARG, "the correction network works on d = 3 plans");
    if (p.geo.Nf < net.n) return fail(ASDSM_E_ARG, "the plan's fine mesh is smaller than the network's volume");
    net.plan = plan;
    net.plan_serial = p.serial;
    net.Nf = p.geo.Nf;
    net.nsp = p.geo.n;
    double am = 0.0;
    for (int j = 0; j < 3; ++j) am += p.alpha[j] / 3.0;
    net.h2a = p.h * p.h / am;
    double centre = 0.0;
    for (int j = 0; j < 3; ++j) {
        net.pe[j] = (float)(p.beta[j] * p.h / (2.0 * p.alpha[j]));
        const Tri &t = p.geo.fine[j];
        centre += t.b;
        net.K.c[1 + 2 * j] = (float)(t.a * net.h2a);  // neighbour i - 1
        net.K.c[2 + 2 * j] = (float)(t.c * net.h2a);  // neighbour i + 1
        net.KT.c[1 + 2 * j] = net.K.c[2 + 2 * j];
        net.KT.c[2 + 2 * j] = net.K.c[1 + 2 * j];
    }
    net.K.c[0] = net.KT.c[0] = (float)(centre * net.h2a);
    set_error("");
    return ASDSM_OK;
}

int asdsm_net_features(asdsm_net_t h, const double *r, double rnorm2, const int *offset, float *in16, float *rhat) {
    if (!h || !r || !in16) return fail(ASDSM_E_ARG, "net, r and in16 must be non-NULL");
    Net &net = h->net;
    if (int rc = require_ws(net)) return rc;
    if (!net.plan) return fail(ASDSM_E_ARG, "the network is not bound to a plan");
    int off[3] = {0, 0, 0};
    for (int j = 0; j < 3; ++j) {
        off[j] = offset ? offset[j] : 0;
        if (off[j] < 0 || off[j] + net.n > net.Nf) return fail(ASDSM_E_ARG, "window outside the fine mesh");
    }
    if (!(rnorm2 >= 0.0) || !std::isfinite(rnorm2)) return fail(ASDSM_E_ARG, "rnorm2 must be finite and >= 0");
    net_features(net.n, net.Nf, net.nsp, off, r, nullptr, rnorm2, net.pe, in16, rhat, nullptr, net.stream);
    NET_HIP_CHECK(hipGetLastError());
    set_error("");
    return ASDSM_OK;
}

int asdsm_net_adam(asdsm_net_t h, float lr) {
    if (!h) return fail(ASDSM_E_ARG, "net must be non-NULL");
    Net &net = h->net;
    if (int rc = require_ws(net)) return rc;
    if (!(lr > 0.f)) return fail(ASDSM_E_ARG, "lr must be positive");
    net.adam_t += 1;
    const float b1 = 0.9f, b2 = 0.999f;
    const float c1 = 1.f - std::pow(b1, (float)net.adam_t), c2 = 1.f - std::pow(b2, (float)net.adam_t);
    net_adam((int)net.nparam, net.P, net.G, net.M, net.V, lr, b1, b2, 1e-8f, c1, c2, net.stream);
    if (int rc = refresh_bf16(net)) return rc;
    set_error("");
    return ASDSM_OK;
}

void asdsm_net_destroy(asdsm_net_t h) {
    if (!h) return;
    if (h->net.hloss) (void)hipHostFree(h->net.hloss);
    delete h;
}

}  // extern "C"
