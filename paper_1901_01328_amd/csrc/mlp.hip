// Monotone CDF network for the learned-splitter sort, trained on the GPU.
//
//   h1 = r(W1*x + b1), h2 = r(W2 @ h1 + b2), f = W3 . h2 + b3,
//   r(z) = min(max(z, 0), 1), weights kept >= 0 (so f never decreases in x).
// Loss: mean squared error against y = rank/n.  Optimizer: Adam followed by
// projection of the weights onto >= 0.  Parameters: 1153 floats
// [W1(32), b1(32), W2(32x32, W2[o][i] at o*32+i), b2(32), W3(32), b3].
//
// The gradient is computed per workgroup over 256 samples: activations and
// back-propagated errors of the workgroup's samples sit in LDS and every
// parameter's partial sum runs over them in a fixed order; the partials of all
// workgroups are then added in workgroup order, so the result is the same on
// every run.  r'(z) is 1 on the open interval (0, 1) and 0 elsewhere.
#include "kpa_internal.hpp"

namespace kpa {

constexpr int H = 32;
constexpr int NP = KPA_MLP_PARAMS;
constexpr int OFF_W1 = 0, OFF_B1 = 32, OFF_W2 = 64, OFF_B2 = 64 + 1024, OFF_W3 = 64 + 1024 + 32,
              OFF_B3 = 64 + 1024 + 64;
static_assert(OFF_B3 + 1 == NP, "parameter layout");

__device__ __forceinline__ float ramp(float z) { return fminf(fmaxf(z, 0.0f), 1.0f); }
__device__ __forceinline__ float dramp(float z) { return (z > 0.0f && z < 1.0f) ? 1.0f : 0.0f; }

__global__ void __launch_bounds__(BLOCK) k_mlp_training_set(const u64* __restrict__ keys, u64 n,
                                                            u32 S, float* __restrict__ x,
                                                            float* __restrict__ y,
                                                            kpa_pwl_model* __restrict__ model) {
  const u64 kmin = keys[0], kmax = keys[n - 1];
  const double span = (double)(kmax - kmin);
  for (u32 s = blockIdx.x * BLOCK + threadIdx.x; s < S; s += gridDim.x * BLOCK) {
    const u64 i = (u64)s * n / S;
    x[s] = span > 0 ? (float)((double)(keys[i] - kmin) / span) : 0.0f;
    y[s] = (float)((double)i / (double)n);
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    model->kmin = kmin;
    model->kmax = kmax;
    model->n_seg = 0;
    model->reserved = 0;
  }
}

__device__ __forceinline__ float mlp_eval(const float* p, float x) {
  float h1[H];
#pragma unroll
  for (int i = 0; i < H; ++i) h1[i] = ramp(p[OFF_W1 + i] * x + p[OFF_B1 + i]);
  float f = p[OFF_B3];
#pragma unroll 4
  for (int o = 0; o < H; ++o) {
    float z = p[OFF_B2 + o];
#pragma unroll
    for (int i = 0; i < H; ++i) z += p[OFF_W2 + o * H + i] * h1[i];
    f += p[OFF_W3 + o] * ramp(z);
  }
  return f;
}

__global__ void __launch_bounds__(BLOCK) k_mlp_forward(const float* __restrict__ params,
                                                       const float* __restrict__ x, u32 m,
                                                       float* __restrict__ out) {
  __shared__ float p[NP];
  for (int i = threadIdx.x; i < NP; i += BLOCK) p[i] = params[i];
  __syncthreads();
  for (u32 s = blockIdx.x * BLOCK + threadIdx.x; s < m; s += gridDim.x * BLOCK)
    out[s] = mlp_eval(p, x[s]);
}

struct GradSmem {
  float p[NP];
  float x[BLOCK];
  float z1[BLOCK][H + 1];  // pre-activations of layer 1 (then dz1)
  float h1[BLOCK][H + 1];
  float z2[BLOCK][H + 1];  // pre-activations of layer 2 (then dz2)
  float df[BLOCK];
  float red[WAVES];
};

// Per-workgroup partial gradient over samples [blk*256, blk*256+256).
__global__ void __launch_bounds__(BLOCK) k_mlp_grad(const float* __restrict__ params,
                                                    const float* __restrict__ x,
                                                    const float* __restrict__ y, u32 m,
                                                    float* __restrict__ partial) {
  __shared__ GradSmem sm;
  const u32 t = threadIdx.x;
  for (int i = t; i < NP; i += BLOCK) sm.p[i] = params[i];
  __syncthreads();
  const u32 s = blockIdx.x * BLOCK + t;
  const bool live = s < m;
  const float xs = live ? x[s] : 0.0f;
  sm.x[t] = xs;
  // forward for this thread's sample
  float f = sm.p[OFF_B3];
#pragma unroll
  for (int i = 0; i < H; ++i) {
    const float z = sm.p[OFF_W1 + i] * xs + sm.p[OFF_B1 + i];
    sm.z1[t][i] = z;
    sm.h1[t][i] = ramp(z);
  }
  for (int o = 0; o < H; ++o) {
    float z = sm.p[OFF_B2 + o];
#pragma unroll
    for (int i = 0; i < H; ++i) z += sm.p[OFF_W2 + o * H + i] * sm.h1[t][i];
    sm.z2[t][o] = z;
    f += sm.p[OFF_W3 + o] * ramp(z);
  }
  const float r = live ? f - y[s] : 0.0f;
  const float df = live ? 2.0f * r / (float)m : 0.0f;
  sm.df[t] = df;
  // loss partial: sum of r^2 / m over the block (fixed order)
  float l = r * r;
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) l += __shfl_xor(l, o, 64);
  if (__lane_id() == 0) sm.red[t >> 6] = l;
  __syncthreads();
  // gW3[o] = sum_s df h2[s][o]; gb3 = sum_s df  (threads 0..32)
  float* out = partial + (u64)blockIdx.x * (NP + 1);
  if (t < H) {
    float g = 0.0f;
    for (int q = 0; q < BLOCK; ++q) g += sm.df[q] * ramp(sm.z2[q][t]);
    out[OFF_W3 + t] = g;
  } else if (t == H) {
    float g = 0.0f;
    for (int q = 0; q < BLOCK; ++q) g += sm.df[q];
    out[OFF_B3] = g;
  } else if (t == H + 1) {
    out[NP] = (sm.red[0] + sm.red[1] + sm.red[2] + sm.red[3]) / (float)m;
  }
  __syncthreads();  // gW3 has read every row of z2
  // dz2[s][o] = df[s] * W3[o] * r'(z2)
  for (int o = 0; o < H; ++o) sm.z2[t][o] = df * sm.p[OFF_W3 + o] * dramp(sm.z2[t][o]);
  __syncthreads();
  // gW2[o][i] = sum_s dz2[s][o] h1[s][i]; 1024 entries, 4 per thread
  for (int e = t; e < H * H; e += BLOCK) {
    const int o = e / H, i = e % H;
    float g = 0.0f;
    for (int q = 0; q < BLOCK; ++q) g += sm.z2[q][o] * sm.h1[q][i];
    out[OFF_W2 + e] = g;
  }
  if (t < H) {
    float g = 0.0f;
    for (int q = 0; q < BLOCK; ++q) g += sm.z2[q][t];
    out[OFF_B2 + t] = g;
  }
  // dz1[s][i] = (sum_o dz2[s][o] W2[o][i]) * r'(z1)
  for (int i = 0; i < H; ++i) {
    float d = 0.0f;
#pragma unroll
    for (int o = 0; o < H; ++o) d += sm.z2[t][o] * sm.p[OFF_W2 + o * H + i];
    sm.z1[t][i] = d * dramp(sm.z1[t][i]);
  }
  __syncthreads();
  if (t < H) {
    float gw = 0.0f, gb = 0.0f;
    for (int q = 0; q < BLOCK; ++q) {
      gw += sm.z1[q][t] * sm.x[q];
      gb += sm.z1[q][t];
    }
    out[OFF_W1 + t] = gw;
    out[OFF_B1 + t] = gb;
  }
}

// Sum of the workgroup partials, in workgroup order (one thread per value).
__global__ void __launch_bounds__(BLOCK) k_mlp_grad_sum(const float* __restrict__ partial,
                                                        u32 nblk, float* __restrict__ grad,
                                                        float* __restrict__ loss) {
  const u32 e = blockIdx.x * BLOCK + threadIdx.x;
  if (e > (u32)NP) return;
  float g = 0.0f;
  for (u32 b = 0; b < nblk; ++b) g += partial[(u64)b * (NP + 1) + e];
  if (e < (u32)NP) grad[e] = g;
  else if (loss) *loss = g;
}

__global__ void __launch_bounds__(BLOCK) k_mlp_adam(float* __restrict__ p, const float* __restrict__ g,
                                                    float* __restrict__ m1, float* __restrict__ v1,
                                                    u32 t, float lr, float b1, float b2, float eps) {
  const int e = blockIdx.x * BLOCK + threadIdx.x;
  if (e >= NP) return;
  const float gi = g[e];
  const float m = b1 * m1[e] + (1.0f - b1) * gi;
  const float v = b2 * v1[e] + (1.0f - b2) * gi * gi;
  m1[e] = m;
  v1[e] = v;
  const float mh = m / (1.0f - powf(b1, (float)t));
  const float vh = v / (1.0f - powf(b2, (float)t));
  float w = p[e] - lr * mh / (sqrtf(vh) + eps);
  const bool is_weight = e < OFF_B1 || (e >= OFF_W2 && e < OFF_B2) || (e >= OFF_W3 && e < OFF_B3);
  if (is_weight) w = fmaxf(w, 0.0f);
  p[e] = w;
}

// Starting parameters from caller-supplied uniforms u in [0, 1) (one per
// parameter; the last is unused): the first layer's ramps get slopes in
// [4, 8) and breakpoints spread over [0, 1] (one per 1/32 interval), the
// second layer starts near an average of its inputs, the output near their
// mean; all weights nonnegative.
__global__ void __launch_bounds__(BLOCK) k_mlp_init(const float* __restrict__ u,
                                                    float* __restrict__ p) {
  const int e = blockIdx.x * BLOCK + threadIdx.x;
  if (e >= NP) return;
  float v;
  if (e < OFF_B1) {
    v = 4.0f + 4.0f * u[e];
  } else if (e < OFF_W2) {
    const int i = e - OFF_B1;
    v = -(4.0f + 4.0f * u[i]) * (((float)i + u[OFF_B1 + i]) / (float)H);
  } else if (e < OFF_B2) {
    v = (0.5f + u[e]) / (float)H;
  } else if (e < OFF_W3) {
    v = -0.25f + 0.5f * u[e];
  } else if (e < OFF_B3) {
    v = (0.5f + u[e]) / (float)H;
  } else {
    v = 0.0f;
  }
  p[e] = v;
}

// Knots of the network's CDF at x = j / S: clamp to [0, 1], running maximum.
__global__ void __launch_bounds__(1024) k_mlp_to_pwl(const float* __restrict__ params, u32 S,
                                                     kpa_pwl_model* __restrict__ model) {
  __shared__ float p[NP];
  __shared__ float wmax[16];
  for (int i = threadIdx.x; i < NP; i += 1024) p[i] = params[i];
  __syncthreads();
  // S + 1 <= 1025 knots: thread j handles knot j (thread 1024 would be knot
  // 1024, so the last thread takes both 1023 and 1024 when S == 1024)
  const u32 j = threadIdx.x;
  float v = j <= S ? ramp(mlp_eval(p, (float)j / (float)S)) : 0.0f;
  float extra = 0.0f;
  if (j == 1023 && S == 1024) extra = ramp(mlp_eval(p, 1.0f));
  // inclusive max scan over 1024 threads
  float sv = v;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const float q = __shfl_up(sv, o, 64);
    if (__lane_id() >= (u32)o) sv = fmaxf(sv, q);
  }
  if (__lane_id() == 63) wmax[threadIdx.x >> 6] = sv;
  __syncthreads();
  for (u32 w = 0; w < (threadIdx.x >> 6); ++w) sv = fmaxf(sv, wmax[w]);
  if (j <= S) model->knots[j] = sv;
  if (j == 1023 && S == 1024) model->knots[1024] = fmaxf(sv, extra);
  if (j == 0) model->n_seg = S;
}

}  // namespace kpa

using namespace kpa;

extern "C" {

kpa_status kpa_mlp_training_set(const uint64_t* sorted_keys, uint64_t n, uint32_t S, float* x,
                                float* y, kpa_pwl_model* out_model, hipStream_t stream) {
  clear_error();
  KPA_REQUIRE(n > 0 && S > 0, KPA_EINVAL, "n and S must be positive");
  KPA_REQUIRE(sorted_keys && x && y && out_model, KPA_EINVAL, "null pointer");
  KPA_LAUNCH("mlp_training_set", k_mlp_training_set, dim3((u32)std::min<u64>(ceil_div(S, BLOCK), 4096)),
             dim3(BLOCK), 0, stream, sorted_keys, n, S, x, y, out_model);
  return KPA_OK;
}

kpa_status kpa_mlp_forward(const float* params, const float* x, uint32_t m, float* out_f,
                           hipStream_t stream) {
  clear_error();
  if (m == 0) return KPA_OK;
  KPA_REQUIRE(params && x && out_f, KPA_EINVAL, "null pointer");
  KPA_LAUNCH("mlp_forward", k_mlp_forward, dim3((u32)std::min<u64>(ceil_div(m, BLOCK), 4096)),
             dim3(BLOCK), 0, stream, params, x, m, out_f);
  return KPA_OK;
}

kpa_status kpa_mlp_loss_grad_workspace_size(uint32_t m, size_t* bytes) {
  clear_error();
  KPA_REQUIRE(bytes, KPA_EINVAL, "bytes is null");
  *bytes = ceil_div(m ? m : 1, BLOCK) * (NP + 1) * sizeof(float) + 256;
  return KPA_OK;
}

static kpa_status loss_grad(const float* params, const float* x, const float* y, uint32_t m,
                            float* out_loss, float* out_grad, void* ws, hipStream_t stream) {
  const u32 nblk = (u32)ceil_div(m, BLOCK);
  float* partial = static_cast<float*>(ws);
  KPA_LAUNCH("mlp_grad", k_mlp_grad, dim3(nblk), dim3(BLOCK), 0, stream, params, x, y, m, partial);
  KPA_LAUNCH("mlp_grad_sum", k_mlp_grad_sum, dim3((u32)ceil_div(NP + 1, BLOCK)), dim3(BLOCK), 0,
             stream, partial, nblk, out_grad, out_loss);
  return KPA_OK;
}

kpa_status kpa_mlp_loss_grad(const float* params, const float* x, const float* y, uint32_t m,
                             float* out_loss, float* out_grad, void* ws, size_t ws_bytes,
                             hipStream_t stream) {
  clear_error();
  KPA_REQUIRE(m > 0, KPA_EINVAL, "m must be positive");
  KPA_REQUIRE(params && x && y && out_grad && ws, KPA_EINVAL, "null pointer");
  size_t need = 0;
  kpa_mlp_loss_grad_workspace_size(m, &need);
  KPA_REQUIRE(ws_bytes >= need, KPA_EWORKSPACE, "workspace too small: need %zu bytes", need);
  return loss_grad(params, x, y, m, out_loss, out_grad, ws, stream);
}

kpa_status kpa_mlp_adam_step(float* params, const float* grad, float* adam_m, float* adam_v,
                             uint32_t t, float lr, float beta1, float beta2, float eps,
                             hipStream_t stream) {
  clear_error();
  KPA_REQUIRE(t >= 1, KPA_EINVAL, "step number starts at 1");
  KPA_REQUIRE(params && grad && adam_m && adam_v, KPA_EINVAL, "null pointer");
  KPA_LAUNCH("mlp_adam", k_mlp_adam, dim3((u32)ceil_div(NP, BLOCK)), dim3(BLOCK), 0, stream, params,
             grad, adam_m, adam_v, t, lr, beta1, beta2, eps);
  return KPA_OK;
}

kpa_status kpa_mlp_train(float* params, float* adam_m, float* adam_v, const float* x,
                         const float* y, uint32_t m, uint32_t t0, uint32_t steps, float lr,
                         float* out_loss, void* ws, size_t ws_bytes, hipStream_t stream) {
  clear_error();
  KPA_REQUIRE(m > 0 && t0 >= 1, KPA_EINVAL, "m must be positive, t0 >= 1");
  KPA_REQUIRE(params && adam_m && adam_v && x && y && ws, KPA_EINVAL, "null pointer");
  size_t need = 0;
  kpa_mlp_loss_grad_workspace_size(m, &need);
  need += NP * sizeof(float) + 256;
  KPA_REQUIRE(ws_bytes >= need, KPA_EWORKSPACE, "workspace too small: need %zu bytes", need);
  Carver c(ws);
  float* partial = c.take<float>(ceil_div(m, BLOCK) * (NP + 1));
  float* grad = c.take<float>(NP);
  for (u32 i = 0; i < steps; ++i) {
    KPA_CHECK(loss_grad(params, x, y, m, i + 1 == steps ? out_loss : nullptr, grad, partial, stream));
    KPA_LAUNCH("mlp_adam", k_mlp_adam, dim3((u32)ceil_div(NP, BLOCK)), dim3(BLOCK), 0, stream, params,
               grad, adam_m, adam_v, t0 + i, lr, 0.9f, 0.999f, 1e-8f);
  }
  return KPA_OK;
}

kpa_status kpa_mlp_init(const float* uniforms, float* params, hipStream_t stream) {
  clear_error();
  KPA_REQUIRE(uniforms && params, KPA_EINVAL, "null pointer");
  KPA_LAUNCH("mlp_init", k_mlp_init, dim3((u32)ceil_div(NP, BLOCK)), dim3(BLOCK), 0, stream,
             uniforms, params);
  return KPA_OK;
}

kpa_status kpa_mlp_to_pwl(const float* params, uint32_t n_seg_model, kpa_pwl_model* model,
                          hipStream_t stream) {
  clear_error();
  KPA_REQUIRE(n_seg_model >= 1 && n_seg_model <= KPA_PWL_MAX_SEG, KPA_EUNSUPPORTED,
              "n_seg_model must be in [1, %d]", KPA_PWL_MAX_SEG);
  KPA_REQUIRE(params && model, KPA_EINVAL, "null pointer");
  KPA_LAUNCH("mlp_to_pwl", k_mlp_to_pwl, dim3(1), dim3(1024), 0, stream, params, n_seg_model, model);
  return KPA_OK;
}

}  // extern "C"
