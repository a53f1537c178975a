// Learned gauge-covariant smoother: parallel-transport convolution layers,
// their gradients, Adam training, and the V-cycle hook.
#pragma once
#include "lib.h"

namespace mgm {

constexpr int kNetMaxLayers = MGM_NET_MAX_LAYERS;
constexpr int kNetMaxWidth = 16;
constexpr int kNetPaths = 9;

struct Net {
  Context* ctx = nullptr;
  const FineOp* op = nullptr;
  mgm_net_desc desc{};
  int L = 0;
  int width[kNetMaxLayers + 1] = {};
  int64_t woff[kNetMaxLayers + 1] = {};  // complex-weight offset of each layer
  int64_t nw = 0;
  double2* w64 = nullptr;   // master weights [nw]
  double2* g64 = nullptr;   // gradient [nw]
  double2* m = nullptr;     // Adam first moment (re, im as separate parameters)
  double2* v = nullptr;     // Adam second moment
  float2* w32 = nullptr;    // kernel weights [layer][path][c_out][c_in]
  float2* wadj = nullptr;   // backward weights [layer][path][c_in][c_out] = W_{opposite path}^H
  float2* buf[2] = {nullptr, nullptr};  // apply ping-pong, 16 channels x max_nrhs
  // training
  float2* act[kNetMaxLayers + 1] = {};  // layer outputs at train_nrhs (act[0] = inputs)
  float2* gbuf[2] = {nullptr, nullptr};
  float2* tr_e = nullptr;   // targets
  double2* wpart = nullptr; // weight-gradient block partials
  int64_t wpart_blocks = 0;
  double* n2 = nullptr;     // [train_nrhs]
  double* e2 = nullptr;
  double* scale = nullptr;
  double* loss = nullptr;   // [1]
  double* pinned = nullptr; // host staging (pinned)
  Scratch scratch;          // reduction partials of the loss norms
  int64_t adam_step = 0;

  void layout(Arena& a);
  void upload_weights(const std::vector<double>& host);  // interleaved complex
  void refresh();          // FP32 copies from the master weights
  // y = N(r), nrhs <= max_nrhs (FP32 fine vectors)
  void apply(const float2* r, float2* y, int nrhs);
  // loss and gradient (into g64) for nrhs <= train_nrhs pairs; returns the loss
  double loss_grad(const float2* r, const float2* e, int nrhs);
  void adam(double lr, double b1, double b2, double eps);
};

// seeded initial weights (host, interleaved complex)
std::vector<double> net_initial_weights(const Net& n, uint64_t seed);

// e = N(r) on the fine level (F32 vectors), used by the V-cycle
void net_apply(Hier& H, Net& net, Vec r, Vec e);

// full-batch Adam training on pairs generated with hierarchy H
void net_train(Hier& H, Net& net, const mgm_train_desc& d, mgm_train_stats* st, double* history);

}  // namespace mgm

struct mgm_net_s {
  mgm::Net n;
  mgm_operator op = nullptr;
};
