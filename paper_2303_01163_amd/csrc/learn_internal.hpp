// Learned correction network: launchers (k_learn.hip) and the network object (net.cpp).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <vector>

namespace asdsm {

// Blocks of the weight-gradient kernel (each sums a fixed set of voxel tiles); the workspace holds
// the partial weight and bias gradients of every block.
constexpr int kNetMaxReduceBlocks = 512;
unsigned net_reduce_blocks(int n);

// 7-point stencil: coefficients of the centre and of the x-, x+, y-, y+, z-, z+ neighbours.
struct NetStencil {
    float c[7];
};

void net_conv_prepare();  // once per process, before the first convolution
void net_conv_fwd(int n, int cin_p, int cout, int cop, bool relu, const void *x, bool x_bf16, const unsigned short *w,
                  const float *bias, void *out, bool out_bf16, const int *gate, hipStream_t st);
void net_conv_wgrad(int n, int cin_p, int cout_p, const float *g, int cop_g, const void *x, bool x_bf16,
                    float *partial, float *dwb, hipStream_t st);
void net_flip(const float *w, int cout_p, int cin_p, unsigned short *wt, hipStream_t st);
void net_to_bf16(const float *a, unsigned short *b, int len, hipStream_t st);
void net_relu_mask(long long nvox, int cop, int cout, const unsigned short *y, float *g, hipStream_t st);
void net_stencil_loss(int n, const float *o, const float *t, const NetStencil &K, const NetStencil &KT, float *rho,
                      float *d16, double *partial, hipStream_t st);
void net_features(int n, int Nf, int nsp, const int off[3], const double *r, const double *rn2, double rn2_value,
                  const float pe[3], float *in16, float *rhat, const int *gate, hipStream_t st);
void net_correction(long long nv, const float *o, const double *rn2, double h2a, double *e, const int *gate,
                    hipStream_t st);
void net_accept(const double *scal, int *done, int *accepted, double factor, int *skip, hipStream_t st);
void net_adam(int len, float *w, const float *g, float *m, float *v, float lr, float b1, float b2, float eps,
              float c1, float c2, hipStream_t st);

// Four 3x3x3 convolutions: 16 (padded input) -> 32 -> 32 -> 32 -> 1, ReLU after the first three.
constexpr int kNetLayers = 4;
constexpr int kNetCinP[kNetLayers] = {16, 32, 32, 32};   // stored input channels
constexpr int kNetCout[kNetLayers] = {32, 32, 32, 1};    // real output channels
constexpr int kNetCoutP[kNetLayers] = {32, 32, 32, 16};  // padded output channels of the weights
constexpr int kNetInputChannels = 7;                     // real input channels (of the 16 stored)

struct Net {
    uint64_t serial = 0;  // unique per network object (never 0)
    int n = 0;
    hipStream_t stream = nullptr;
    long long nvox = 0;
    size_t wofs[kNetLayers] = {}, bofs[kNetLayers] = {};  // offsets in the flat parameter vector
    size_t nparam = 0;
    std::vector<float> host_params;                       // initial values until the workspace exists
    int adam_t = 0;
    // device buffers (inside the caller's workspace)
    void *ws = nullptr;
    size_t ws_need = 0;
    float *P = nullptr, *G = nullptr, *M = nullptr, *V = nullptr;
    unsigned short *Wb[kNetLayers] = {};
    unsigned short *Wt = nullptr;
    // act[0] = input copy (16 ch, FP32), act[1..3] (32 ch, stored BF16), act[4] output (1 ch, FP32)
    float *act[kNetLayers + 1] = {};
    float *gA = nullptr, *gB = nullptr, *d16 = nullptr, *target = nullptr;
    float *partial = nullptr;
    float *rho = nullptr;     // residual of the loss (n^3)
    double *lpart = nullptr;
    int *skip = nullptr;      // flags of the acceptance test (two ints)
    double *hloss = nullptr;  // pinned
    int nblk_loss = 0;
    // binding to a plan (d = 3): features and the operator of the residual loss
    const void *plan = nullptr;
    uint64_t plan_serial = 0;
    int Nf = 0, nsp = 0;
    float pe[3] = {};
    double h2a = 0.0;         // h^2 / mean(alpha)
    NetStencil K = {}, KT = {};
};

}  // namespace asdsm

struct asdsm_net_s {
    asdsm::Net net;
};
