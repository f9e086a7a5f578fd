// Predictions of repeated gate applications and the statistical distance.
//
// Thesis Eq. GSTPrediction: p_r = <<E_m| (G_s)^r G_prep |rho>> for r = 0 .. r_max,
// for preparation words G_prep and gates s.  The powers are evaluated in
// blocks of B = 2^(levels-1) repetitions: predict_chain_kernel applies the
// preparation word to rho, builds (G_s)^B in LDS by repeated squaring and
// steps from one block start to the next with it; predict_fill_kernel then
// runs each block with single steps and reads out every state.  The first
// block is the plain evaluation step for step (bit-identical probabilities);
// later blocks start from states that carry the rounding of the matrix power.
// Eq. statisticaldistance: D = 1/2 sum_m |p_m - q_m| per row.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "gst_device.h"
#include "gst_internal.h"

namespace gst {
namespace {

__host__ __device__ inline size_t predict_head_doubles(int K) {
  return (size_t)2 * K * GATE_STRIDE + 2 * 16 * ROW + 16;
}

// One single-wave workgroup per (preparation, gate) pair.
template <int D>
__global__ __launch_bounds__(64) void predict_chain_kernel(const PredictLaunch a) {
  extern __shared__ double lds_raw[];
  const int K = a.K;
  const Lds s = carve(lds_raw, K);
  const int lane = threadIdx.x & 63, i = lane & 15;
  stage_gateset<D, 64, STAGE_G>(s, a.G, a.E, a.rho, K, a.M);
  double* js = lds_raw + predict_head_doubles(K);
  for (int pair = blockIdx.x; pair < a.n_pairs; pair += gridDim.x) {
    const int p = pair / a.n_gates, g = a.gate_of[pair % a.n_gates];
    // the preparation word (at most 64 gates; lane j holds gate j)
    const int64_t x0 = a.prep_off[p], L = a.prep_off[p + 1] - x0;
    const int kw = lane < L ? (int)a.prep_gates[x0 + lane] : 0;
    double f = s.rho[i];
    for (int x = 0; x < (int)L; ++x) {
      const int k = __builtin_amdgcn_readlane(kw, x);
      f = dot16(f, load_row(s.Gs + k * GATE_STRIDE + i * ROW));
    }
    build_jumps(js, s.Gs, 1u | (uint32_t)g << 8, 0, a.levels, false, lane);
    const Row16 RJ = load_row(js + (a.levels - 1) * GATE_STRIDE + i * ROW);
    double* v = a.V + (int64_t)pair * a.Q * D;
    if (lane < D) v[i] = f;
    for (int q = 1; q < a.Q; ++q) {
      f = dot16(f, RJ);
      if (lane < D) v[(int64_t)q * D + i] = f;
    }
    wave_sync();  // js is rebuilt for the next pair
  }
}

// One 16-lane team per (pair, block): B single steps from the block's start
// state, the readout of every state before the step.
template <int D>
__global__ __launch_bounds__(256) void predict_fill_kernel(const PredictLaunch a) {
  extern __shared__ double lds_raw[];
  const int K = a.K, M = a.M;
  const Lds s = carve(lds_raw, K);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, i = lane & 15, team = lane >> 4;
  stage_gateset<D, 256, STAGE_G | STAGE_E>(s, a.G, a.E, a.rho, K, M);
  const Row16 ER = load_row(s.Es + i * ROW);
  const int64_t n_tasks = (int64_t)a.n_pairs * a.Q;
  const int64_t n_groups = (n_tasks + TPW - 1) / TPW;
  const int B = 1 << (a.levels - 1);
  for (int64_t grp = (int64_t)blockIdx.x * WAVES + wave; grp < n_groups; grp += (int64_t)gridDim.x * WAVES) {
    const int64_t t = grp * TPW + team;
    const bool has = t < n_tasks;
    const int64_t pair = has ? t / a.Q : 0;
    const int q = has ? (int)(t % a.Q) : 0;
    const int g = a.gate_of[pair % a.n_gates];
    const Row16 R = load_row(s.Gs + g * GATE_STRIDE + i * ROW);
    double f = i < D ? a.V[(pair * a.Q + q) * D + i] : 0.0;
    double* out = a.probs + pair * (int64_t)(a.r_max + 1) * M;
    for (int k = 0; k < B; ++k) {
      const int r = q * B + k;
      const double pm = dot16(f, ER);
      if (has && i < M && r <= a.r_max) out[(int64_t)r * M + i] = pm;
      if (k + 1 < B) f = dot16(f, R);
    }
  }
}

__global__ __launch_bounds__(256) void tv_distance_kernel(const double* __restrict__ p, const double* __restrict__ q,
                                                          int64_t n, int M, double* __restrict__ out) {
  for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < n; r += (int64_t)gridDim.x * blockDim.x) {
    double acc = 0.0;
    for (int m = 0; m < M; ++m) acc += fabs(p[r * M + m] - q[r * M + m]);
    out[r] = 0.5 * acc;
  }
}

}  // namespace

static bool predict_args_ok(const PredictLaunch& a) {
  return a.n_pairs > 0 && a.Q > 0 && a.levels >= 1 && a.levels <= 6 && (a.D == 4 || a.D == 16);
}

hipError_t launch_predict_chain(const PredictLaunch& a, hipStream_t stream) {
  if (!predict_args_ok(a)) return hipErrorInvalidValue;
  const size_t bytes = (predict_head_doubles(a.K) + (size_t)a.levels * GATE_STRIDE) * 8 + 64;
  const int blocks = a.n_pairs < 65535 ? a.n_pairs : 65535;
  if (a.D == 16)
    gst_launch(predict_chain_kernel<16>, dim3(blocks), dim3(64), bytes, stream, a);
  else
    gst_launch(predict_chain_kernel<4>, dim3(blocks), dim3(64), bytes, stream, a);
  return hipGetLastError();
}

hipError_t launch_predict_fill(const PredictLaunch& a, hipStream_t stream) {
  if (!predict_args_ok(a)) return hipErrorInvalidValue;
  const size_t bytes = predict_head_doubles(a.K) * 8 + 64;
  const int64_t groups = ((int64_t)a.n_pairs * a.Q + TPW - 1) / TPW;
  const int64_t want = (groups + WAVES - 1) / WAVES;
  const int blocks = (int)(want < 4096 ? want : 4096);
  if (a.D == 16)
    gst_launch(predict_fill_kernel<16>, dim3(blocks), dim3(256), bytes, stream, a);
  else
    gst_launch(predict_fill_kernel<4>, dim3(blocks), dim3(256), bytes, stream, a);
  return hipGetLastError();
}

hipError_t launch_tv_distance(const double* p, const double* q, int64_t n, int M, double* out, hipStream_t stream) {
  if (n <= 0) return hipSuccess;
  const int64_t b = (n + 255) / 256;
  gst_launch(tv_distance_kernel, dim3((unsigned)(b < 65535 ? b : 65535)), dim3(256), 0, stream, p, q, n, M, out);
  return hipGetLastError();
}

}  // namespace gst
