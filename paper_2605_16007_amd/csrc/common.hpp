// Shared helpers of librbq: status plumbing and order-preserving sort keys.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <stdexcept>
#include <string>

#include "rbq.h"

namespace rbq {

// An error that crosses back to the C ABI as a status plus message.
struct Error : std::runtime_error {
  rbq_status status;
  Error(rbq_status s, const std::string& m) : std::runtime_error(m), status(s) {}
};

[[noreturn]] inline void fail(rbq_status s, const std::string& m) { throw Error(s, m); }

#define RBQ_HIP(call)                                                                       \
  do {                                                                                      \
    hipError_t e_ = (call);                                                                 \
    if (e_ != hipSuccess)                                                                   \
      ::rbq::fail(e_ == hipErrorOutOfMemory ? RBQ_ENOMEM : RBQ_EDEVICE,                     \
                  std::string(#call) + ": " + hipGetErrorString(e_));                       \
  } while (0)

#define RBQ_CHECK(cond, msg)                        \
  do {                                              \
    if (!(cond)) ::rbq::fail(RBQ_EINVAL, (msg));    \
  } while (0)

// Order-preserving map float -> uint32 (ascending floats give ascending keys;
// -0.0 sorts just below +0.0). Selection runs on 64-bit keys
// (ordered value << 32 | tie), so ties break by the low word.
__host__ __device__ inline uint32_t ord_f32(float f) {
  uint32_t u;
  __builtin_memcpy(&u, &f, 4);
  return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}
__host__ __device__ inline float f32_ord(uint32_t o) {
  uint32_t u = (o & 0x80000000u) ? (o & 0x7fffffffu) : ~o;
  float f;
  __builtin_memcpy(&f, &u, 4);
  return f;
}
__host__ __device__ inline uint64_t key64(float v, uint32_t tie) {
  return (static_cast<uint64_t>(ord_f32(v)) << 32) | tie;
}
constexpr uint64_t KEY_NONE = ~0ull;

// d_hat^2 of Eq. approx-dist from the exact integer inner product
// ip = sum_d b01_d qu_d (Eq. rabitq-ip-estimator with the B_q-bit query):
//   d_hat^2 = ||r||^2 + n_x^2 + f_x E,  f_x = -2 n_x / (sqrt(D) alpha_x),
//   E = v_l (2 pop - D) + Delta (2 ip - sum qu),
// regrouped as fma(f_x Delta, 2 ip - sum qu, fma(v_l, vx, n_x^2)) + ||r||^2
// with the per-vector vx = f_x (2 pop - D). Every scan evaluates exactly this
// expression, so their estimates agree bit for bit.
__device__ __forceinline__ float rbq_vx(float fmul, int pop, int D) {
  return fmul * (float)(2 * pop - D);
}
// The estimate without its last term ||r||^2, from g = 2 ip - sum qu as a
// float that holds the integer exactly (|g| < 2^24), as a float-accumulating
// matrix core returns it; d_hat^2 = part + ||r||^2.
__device__ __forceinline__ float rbq_estimate_part(float vl, float delta, float g, float fadd, float fmul,
                                                   float vx) {
  return __builtin_fmaf(fmul * delta, g, __builtin_fmaf(vl, vx, fadd));
}
__device__ __forceinline__ float rbq_estimate_gf(float rn2, float vl, float delta, float g, float fadd,
                                                 float fmul, float vx) {
  return rbq_estimate_part(vl, delta, g, fadd, fmul, vx) + rn2;
}
// A bound b on the part such that part + ||r||^2 <= thr (rounded to nearest)
// implies part <= b: the sum's rounding error is at most |thr| 2^-24 below
// thr, and the margin (|thr| + ||r||^2) 2^-20 also covers the two roundings
// of b itself. +inf stays +inf; a NaN threshold gives a NaN bound (no part
// passes).
__device__ __forceinline__ float rbq_part_bound(float thr, float rn2) {
  const float m = __builtin_fmaxf((__builtin_fabsf(thr) + __builtin_fabsf(rn2)) * 0x1p-20f, 0x1p-100f);
  return (thr - rn2) + m;
}
// from g = 2 ip - sum qu, an exact integer
__device__ __forceinline__ float rbq_estimate_g(float rn2, float vl, float delta, int g, float fadd,
                                                float fmul, float vx) {
  return rbq_estimate_gf(rn2, vl, delta, (float)g, fadd, fmul, vx);
}
// (neg_sumqu = -sum qu, so that 2 ip - sum qu is one shift-add)
__device__ __forceinline__ float rbq_estimate(float rn2, float vl, float delta, int neg_sumqu, int ip,
                                              float fadd, float fmul, float vx) {
  return rbq_estimate_g(rn2, vl, delta, (ip << 1) + neg_sumqu, fadd, fmul, vx);
}

inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }
inline int64_t round_up(int64_t a, int64_t b) { return ceil_div(a, b) * b; }

}  // namespace rbq
