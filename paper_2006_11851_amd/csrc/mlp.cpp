// Leaf-proposal MLP: parameters, training loop, gradient entry points and
// the matrix-core inference used by the learned search modes.
//
// The network is trained on (PCA query, leaf of its exact match) pairs with
// softmax cross-entropy and Adam; FP32 master weights, GEMM operands in bf16
// (or FP32 for gradient checks).  Minibatches are drawn on the GPU from a
// counter-based hash, so training needs no host round trips except the
// logged losses.
#include <cfloat>
#include <cmath>
#include <cstring>

#include "api_internal.hpp"
#include "kernels_mlp.hpp"

using namespace pts;

namespace pts {

namespace {

struct Layout {
  int64_t W1, b1, W2, b2, W3, b3, total;
};

Layout layout(const Mlp& m) {
  Layout L;
  L.W1 = 0;
  L.b1 = L.W1 + (int64_t)m.h * m.n_in;
  L.W2 = L.b1 + m.h;
  L.b2 = L.W2 + (int64_t)m.h * m.h;
  L.W3 = L.b2 + m.h;
  L.b3 = L.W3 + (int64_t)m.n_out * m.h;
  L.total = L.b3 + m.n_out;
  return L;
}

int k_in(const Mlp& m) { return (int)round_up(m.n_in, 32); }

struct Work {
  float *A0, *Z1, *H1, *Z2, *H2, *L, *G, *dH2, *dH1, *row_loss, *loss;
  int32_t* lab;
  int64_t* idx;
};

Work workspace(Ctx* c, const Mlp& m, int64_t B) {
  Work w;
  w.A0 = c->buf<float>("mlp_A0", (size_t)B * m.n_in);
  w.Z1 = c->buf<float>("mlp_Z1", (size_t)B * m.h);
  w.H1 = c->buf<float>("mlp_H1", (size_t)B * m.h);
  w.Z2 = c->buf<float>("mlp_Z2", (size_t)B * m.h);
  w.H2 = c->buf<float>("mlp_H2", (size_t)B * m.h);
  w.L = c->buf<float>("mlp_L", (size_t)B * m.n_out);
  w.G = c->buf<float>("mlp_G", (size_t)B * m.n_out);
  w.dH2 = c->buf<float>("mlp_dH2", (size_t)B * m.h);
  w.dH1 = c->buf<float>("mlp_dH1", (size_t)B * m.h);
  w.row_loss = c->buf<float>("mlp_row_loss", (size_t)B);
  w.loss = c->buf<float>("mlp_loss", 1);
  w.lab = c->buf<int32_t>("mlp_lab", (size_t)B);
  w.idx = c->buf<int64_t>("mlp_idx", (size_t)B);
  return w;
}

void forward(Ctx* c, const Mlp& m, const float* P, const Work& w, int64_t B, bool bf) {
  const Layout L = layout(m);
  const int Bi = (int)B;
  launch_gemm(c, false, true, bf, w.A0, P + L.W1, w.Z1, Bi, m.h, m.n_in, false);
  launch_bias_act(c, w.Z1, w.H1, P + L.b1, B, m.h, true);
  launch_gemm(c, false, true, bf, w.H1, P + L.W2, w.Z2, Bi, m.h, m.h, false);
  launch_bias_act(c, w.Z2, w.H2, P + L.b2, B, m.h, true);
  launch_gemm(c, false, true, bf, w.H2, P + L.W3, w.L, Bi, m.n_out, m.h, false);
  launch_bias_act(c, w.L, nullptr, P + L.b3, B, m.n_out, false);
}

// loss (device scalar) and gradient (packed, device) of the batch in w
void loss_grad(Ctx* c, const Mlp& m, const float* P, const Work& w, int64_t B, bool bf, float* grad) {
  const Layout L = layout(m);
  const int Bi = (int)B;
  forward(c, m, P, w, B, bf);
  launch_softmax_ce(c, w.L, w.lab, B, m.n_out, w.G, w.row_loss);
  launch_mean(c, w.row_loss, B, w.loss);
  // output layer
  launch_gemm(c, true, false, bf, w.G, w.H2, grad + L.W3, m.n_out, m.h, Bi, false);
  launch_colsum(c, w.G, B, m.n_out, grad + L.b3);
  launch_gemm(c, false, false, bf, w.G, P + L.W3, w.dH2, Bi, m.h, m.n_out, false);
  launch_gelu_bwd(c, w.dH2, w.Z2, B * m.h);
  // second layer
  launch_gemm(c, true, false, bf, w.dH2, w.H1, grad + L.W2, m.h, m.h, Bi, false);
  launch_colsum(c, w.dH2, B, m.h, grad + L.b2);
  launch_gemm(c, false, false, bf, w.dH2, P + L.W2, w.dH1, Bi, m.h, m.h, false);
  launch_gelu_bwd(c, w.dH1, w.Z1, B * m.h);
  // first layer
  launch_gemm(c, true, false, bf, w.dH1, w.A0, grad + L.W1, m.h, m.n_in, Bi, false);
  launch_colsum(c, w.dH1, B, m.h, grad + L.b1);
}

Mlp& require_mlp(Ctx* c) {
  PTS_REQUIRE(c->mlp.valid, PTS_ERR_STATE, "no MLP: call pts_mlp_init first");
  return c->mlp;
}

void mark_changed(Ctx* c) { c->mlp.version++; }

// bf16 weight copies for inference, rebuilt after any weight change
const Mlp& bf_weights(Ctx* c) {
  Mlp& m = c->mlp;
  if (m.bf_version != m.version) {
    const Layout L = layout(m);
    const float* P = m.params.as<float>();
    const int K1 = k_in(m);
    uint16_t* w1 = static_cast<uint16_t*>(m.w1b.ensure(c, (size_t)m.h * K1 * 2));
    uint16_t* w2 = static_cast<uint16_t*>(m.w2b.ensure(c, (size_t)m.h * m.h * 2));
    uint16_t* w3 = static_cast<uint16_t*>(m.w3b.ensure(c, (size_t)round_up(m.n_out, 32) * m.h * 2));
    launch_to_bf16_pad(c, P + L.W1, m.h, m.n_in, m.h, K1, false, w1);
    launch_to_bf16_pad(c, P + L.W2, m.h, m.h, m.h, m.h, true, w2);
    launch_to_bf16_pad(c, P + L.W3, m.n_out, m.h, (int)round_up(m.n_out, 32), m.h, true, w3);
    float* b3p = static_cast<float*>(m.b3p.ensure(c, (size_t)round_up(m.n_out, 32) * 4));
    launch_pad_f32(c, P + L.b3, m.n_out, (int)round_up(m.n_out, 32), -FLT_MAX, b3p);
    m.bf_version = m.version;
  }
  return m;
}

}  // namespace

void mlp_propose_rows(Ctx* c, const float* Qp, int ld, int64_t n, int k, int32_t* leaves, float* margin) {
  Mlp& m = require_mlp(c);
  const Mlp& bc = bf_weights(c);
  const Layout L = layout(m);
  const float* P = m.params.as<float>();
  const int K1 = k_in(m);
  launch_mlp_propose(c, Qp, ld, n, m.in_scale.as<float>(), m.n_in, K1, bc.w1b.as<uint16_t>(), P + L.b1,
                     bc.w2b.as<uint16_t>(), P + L.b2, m.h, bc.w3b.as<uint16_t>(), bc.b3p.as<float>(), m.n_out, k,
                     leaves, margin);
}

}  // namespace pts

// ------------------------------------------------------------------ C ABI

template <class F>
static int mguard(pts_ctx* c, F&& f) {
  if (!c) return PTS_ERR_ARG;
  try {
    PTS_HIP(hipSetDevice(c->device));
    f();
    c->last_error.clear();
    return PTS_OK;
  } catch (const pts::Error& e) {
    c->last_error = e.msg;
    return e.code;
  } catch (const std::bad_alloc&) {
    c->last_error = "host allocation failed";
    return PTS_ERR_OOM;
  }
}

extern "C" {

int pts_mlp_init(pts_ctx* c, int n_in, int hidden, int n_out, uint64_t seed) {
  return mguard(c, [&] {
    PTS_REQUIRE(n_in >= 1 && n_in <= 128, PTS_ERR_UNSUPPORTED, "mlp: n_in must be 1..128");
    PTS_REQUIRE(hidden == 32 || hidden == 64 || hidden == 128 || hidden == 256, PTS_ERR_UNSUPPORTED,
                "mlp: hidden must be 32, 64, 128 or 256");
    PTS_REQUIRE(n_out >= 2 && n_out <= 65536, PTS_ERR_UNSUPPORTED, "mlp: n_out must be 2..65536");
    Mlp& m = c->mlp;
    m.n_in = n_in;
    m.h = hidden;
    m.n_out = n_out;
    const Layout L = layout(m);
    m.n_params = L.total;
    // uniform(-1/sqrt(fan_in), 1/sqrt(fan_in)) for weights and biases
    std::vector<float> p(L.total);
    uint64_t s = seed * 0x9E3779B97F4A7C15ull + 0x632BE59BD9B4E019ull;
    auto uni = [&]() {
      s += 0x9E3779B97F4A7C15ull;
      uint64_t z = s;
      z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
      z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
      z ^= z >> 31;
      return (double)(z >> 11) * (1.0 / 9007199254740992.0) * 2.0 - 1.0;
    };
    auto fill = [&](int64_t off, int64_t n, int fan_in) {
      const double a = 1.0 / std::sqrt((double)fan_in);
      for (int64_t i = 0; i < n; ++i) p[off + i] = (float)(a * uni());
    };
    fill(L.W1, L.b1 - L.W1, n_in);
    fill(L.b1, hidden, n_in);
    fill(L.W2, L.b2 - L.W2, hidden);
    fill(L.b2, hidden, hidden);
    fill(L.W3, L.b3 - L.W3, hidden);
    fill(L.b3, n_out, hidden);
    float* dp = static_cast<float*>(m.params.ensure(c, (size_t)L.total * 4));
    PTS_HIP(hipMemcpyAsync(dp, p.data(), (size_t)L.total * 4, hipMemcpyHostToDevice, c->stream));
    std::vector<float> zero(L.total, 0.f);
    float* am = static_cast<float*>(m.adam_m.ensure(c, (size_t)L.total * 4));
    float* av = static_cast<float*>(m.adam_v.ensure(c, (size_t)L.total * 4));
    PTS_HIP(hipMemcpyAsync(am, zero.data(), (size_t)L.total * 4, hipMemcpyHostToDevice, c->stream));
    PTS_HIP(hipMemcpyAsync(av, zero.data(), (size_t)L.total * 4, hipMemcpyHostToDevice, c->stream));
    m.adam_t = 0;
    // input scale: whiten by the index's eigenvalues when the widths match
    std::vector<float> sc(n_in, 1.f);
    if (c->index.valid && c->index.d == n_in && (int)c->index.eig.size() == n_in)
      for (int k = 0; k < n_in; ++k) sc[k] = (float)(1.0 / std::sqrt(std::max(c->index.eig[k], 1e-12)));
    float* ds = static_cast<float*>(m.in_scale.ensure(c, (size_t)n_in * 4));
    PTS_HIP(hipMemcpyAsync(ds, sc.data(), (size_t)n_in * 4, hipMemcpyHostToDevice, c->stream));
    PTS_HIP(hipStreamSynchronize(c->stream));
    m.valid = true;
    mark_changed(c);
  });
}

int pts_mlp_n_params(pts_ctx* c, int64_t* n) {
  return mguard(c, [&] {
    PTS_REQUIRE(n, PTS_ERR_ARG, "null");
    *n = require_mlp(c).n_params;
  });
}

int pts_mlp_get_weights(pts_ctx* c, float* host) {
  return mguard(c, [&] {
    PTS_REQUIRE(host, PTS_ERR_ARG, "null");
    Mlp& m = require_mlp(c);
    PTS_HIP(hipMemcpyAsync(host, m.params.ptr, (size_t)m.n_params * 4, hipMemcpyDeviceToHost, c->stream));
    PTS_HIP(hipStreamSynchronize(c->stream));
  });
}

int pts_mlp_set_weights(pts_ctx* c, const float* host) {
  return mguard(c, [&] {
    PTS_REQUIRE(host, PTS_ERR_ARG, "null");
    Mlp& m = require_mlp(c);
    PTS_HIP(hipMemcpyAsync(m.params.ptr, host, (size_t)m.n_params * 4, hipMemcpyHostToDevice, c->stream));
    PTS_HIP(hipStreamSynchronize(c->stream));
    mark_changed(c);
  });
}

int pts_mlp_set_input_scale(pts_ctx* c, const float* host) {
  return mguard(c, [&] {
    PTS_REQUIRE(host, PTS_ERR_ARG, "null");
    Mlp& m = require_mlp(c);
    PTS_HIP(hipMemcpyAsync(m.in_scale.ptr, host, (size_t)m.n_in * 4, hipMemcpyHostToDevice, c->stream));
    PTS_HIP(hipStreamSynchronize(c->stream));
  });
}

int pts_mlp_forward(pts_ctx* c, const float* q, int64_t n, int bf16, float* logits) {
  return mguard(c, [&] {
    Mlp& m = require_mlp(c);
    PTS_REQUIRE(n >= 0 && n < (1 << 30) && (n == 0 || (q && logits)), PTS_ERR_ARG, "mlp_forward: bad arguments");
    if (n == 0) return;
    Work w = workspace(c, m, n);
    launch_gather_scale(c, q, m.n_in, m.in_scale.as<float>(), m.n_in, nullptr, nullptr, n, w.A0, nullptr);
    forward(c, m, m.params.as<float>(), w, n, bf16 != 0);
    PTS_HIP(hipMemcpyAsync(logits, w.L, (size_t)n * m.n_out * 4, hipMemcpyDeviceToDevice, c->stream));
  });
}

int pts_mlp_loss_grad(pts_ctx* c, const float* q, const int32_t* label, int64_t n, int bf16, float* grad,
                      float* loss_host) {
  return mguard(c, [&] {
    Mlp& m = require_mlp(c);
    PTS_REQUIRE(n >= 1 && n < (1 << 30) && q && label && grad, PTS_ERR_ARG, "mlp_loss_grad: bad arguments");
    Work w = workspace(c, m, n);
    launch_gather_scale(c, q, m.n_in, m.in_scale.as<float>(), m.n_in, nullptr, label, n, w.A0, w.lab);
    loss_grad(c, m, m.params.as<float>(), w, n, bf16 != 0, grad);
    if (loss_host) {
      PTS_HIP(hipMemcpyAsync(loss_host, w.loss, 4, hipMemcpyDeviceToHost, c->stream));
      PTS_HIP(hipStreamSynchronize(c->stream));
    }
  });
}

int pts_mlp_train(pts_ctx* c, const float* q, const int32_t* label, int64_t n, const pts_train_params* p,
                  float* loss_log) {
  return mguard(c, [&] {
    Mlp& m = require_mlp(c);
    PTS_REQUIRE(p && q && label && n >= 1, PTS_ERR_ARG, "mlp_train: bad arguments");
    PTS_REQUIRE(p->batch >= 1 && p->batch <= (1 << 20) && p->steps >= 0, PTS_ERR_ARG, "mlp_train: bad batch/steps");
    PTS_REQUIRE(p->lr > 0.f && p->beta1 >= 0.f && p->beta1 < 1.f && p->beta2 >= 0.f && p->beta2 < 1.f && p->eps > 0.f,
                PTS_ERR_ARG, "mlp_train: bad Adam parameters");
    const int64_t B = p->batch;
    Work w = workspace(c, m, B);
    float* grad = c->buf<float>("mlp_grad", (size_t)m.n_params);
    const int log_every = p->log_every > 0 ? p->log_every : 0;
    for (int64_t st = 0; st < p->steps; ++st) {
      launch_sample_idx(c, p->seed, st, (int)B, n, w.idx);
      launch_gather_scale(c, q, m.n_in, m.in_scale.as<float>(), m.n_in, w.idx, label, B, w.A0, w.lab);
      loss_grad(c, m, m.params.as<float>(), w, B, p->bf16 != 0, grad);
      m.adam_t += 1;
      launch_adam(c, m.params.as<float>(), grad, m.adam_m.as<float>(), m.adam_v.as<float>(), m.n_params, p->lr,
                  p->beta1, p->beta2, p->eps, m.adam_t);
      if (loss_log && log_every && (st + 1) % log_every == 0) {
        PTS_HIP(hipMemcpyAsync(loss_log + (st + 1) / log_every - 1, w.loss, 4, hipMemcpyDeviceToHost, c->stream));
      }
    }
    PTS_HIP(hipStreamSynchronize(c->stream));
    mark_changed(c);
  });
}

int pts_mlp_propose(pts_ctx* c, const float* q, int64_t n, int k, int32_t* leaves, float* margin) {
  return mguard(c, [&] {
    Mlp& m = require_mlp(c);
    PTS_REQUIRE(n >= 0 && (n == 0 || (q && leaves && margin)), PTS_ERR_ARG, "mlp_propose: bad arguments");
    PTS_REQUIRE(k >= 1 && k <= 8 && k <= m.n_out, PTS_ERR_ARG, "mlp_propose: k must be 1..8");
    if (n) mlp_propose_rows(c, q, m.n_in, n, k, leaves, margin);
  });
}

}  // extern "C"
