// Batched evaluation of many requests in one persistent launch.
//
// Work is cut into tiles; a tile is a run of sequences of ONE request (the
// request's sequences sorted by length, cut into tiles of a size fixed by the
// request alone).  Workgroups take tiles from an atomic queue; the gate set of
// a tile's request is staged into LDS when it differs from the one already
// there.  Every tile writes its own slab of partial sums, and each request's
// slabs are added in tile order afterwards, so a request's results do not
// depend on which workgroup ran which tile, nor on the other requests of the
// batch.
//
// The per-sequence work is that of the plain sequence kernel (forward chain
// with checkpoints, readout, objective, seeds, reverse sweep, dG through the
// LDS stash and MFMA tiles).
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "gst_device.h"
#include "gst_internal.h"

namespace gst {
namespace {

// The slab reduction reuses the LDS of the staged gate set (as in the plain
// sequence kernel), so a workgroup restages after every tile that writes a
// slab; the smaller footprint keeps two or three workgroups per CU.
// The tile index a workgroup works on sits in the last 16 bytes.  (A static
// __shared__ variable would be placed before the dynamic area and shift it
// off the 16-byte alignment that the row reads of ds_read_b128 need.)
__host__ __device__ inline size_t batch_lds_core(int K) {
  const size_t a = lds_main_bytes(K), b = lds_red_bytes(K);
  return ((a > b ? a : b) + 15) / 16 * 16;
}
__host__ __device__ inline size_t batch_lds_bytes(int K) { return batch_lds_core(K) + 16; }

template <int D>
__global__ __launch_bounds__(256) void batch_kernel(const BatchLaunch a) {
  extern __shared__ double lds_raw[];
  int& tile_sh = *reinterpret_cast<int*>(reinterpret_cast<char*>(lds_raw) + batch_lds_core(a.kmax));
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, i = lane & 15, team = lane >> 4;
  int staged = -1;
  Lds s = carve(lds_raw, a.kmax);
  double* st_b = s.stash + (size_t)wave * 2 * ENT * 16;
  double* st_f = st_b + ENT * 16;
  uint8_t* st_k = s.sk + wave * ENT;
  const int64_t gteam = ((int64_t)blockIdx.x * WAVES + wave) * TPW + team;
  double* ck = a.ckpt + gteam * a.ckpt_per_team;
  for (;;) {
    if (tid == 0) tile_sh = (int)atomicAdd(a.queue, 1u);
    __syncthreads();
    const int tile = tile_sh;
    __syncthreads();
    if (tile >= a.n_tiles) break;
    const BatchTile T = a.tiles[tile];
    const BatchReq R = a.reqs ? a.reqs[T.req] : a.one;
    const int K = R.K, M = R.M;
    const auto* g_off = as_global(R.off);
    const auto* g_order = as_global(R.order);
    const auto* g_gates = as_global(R.gates);
    const auto* g_counts = as_global(R.counts);
    const auto* g_W = as_global(R.W);
    auto* g_probs = as_global(R.probs);
    if (T.req != staged) {
      // a different gate set: restage (carve for this request's K inside the kmax layout)
      s = carve(lds_raw, a.kmax);
      stage_gateset_compact<D>(s, R.G, R.E, R.rho, K, M);  // the tile loop is short of registers
      staged = T.req;
    }
    const bool grad = R.want_grad != 0;
    d4 acc[KMAX];
#pragma unroll
    for (int k = 0; k < KMAX; ++k) acc[k] = d4{0.0, 0.0, 0.0, 0.0};
    double obj = 0.0, drho = 0.0;
    double dE[16];
#pragma unroll
    for (int m = 0; m < 16; ++m) dE[m] = 0.0;
    unsigned bad = 0, nonpos = 0;
    const int64_t nq = T.q1 - T.q0;
    const int64_t n_groups = (nq + TPW - 1) / TPW;
    for (int64_t grp = wave; grp < n_groups; grp += WAVES) {
      const int64_t qq = T.q0 + grp * TPW + team;
      const bool has = qq < T.q1;
      const int64_t seq = has ? (R.order ? g_order[qq] : qq) : 0;
      const int64_t beg = has ? g_off[seq] : 0;
      const int L = has ? (int)(g_off[seq + 1] - beg) : 0;
      const int Lw = wave_max4(L);
      const auto* word = g_gates + beg;
      double f = s.rho[i];
      // Gate indices are loaded one chunk of 16 steps ahead of their use.
      // The loads are unconditional (past the end of the word they read the
      // first index of the list, which always exists) so that the compiler
      // can wait for the previous load alone.
      int kv_next = *(i < L ? word + i : g_gates);
      kv_next = i < L ? kv_next : 0;
      for (int t0 = 0; t0 < Lw; t0 += 16) {
        int kv = kv_next;
        const bool in = t0 + 16 + i < L;
        kv_next = *(in ? word + t0 + 16 + i : g_gates);
        kv_next = in ? kv_next : 0;
        if (t0 + i < L && kv >= K) {
          ++bad;
          kv = 0;
        }
#define GST_FWD_STEP(RR)                                                   \
  if (t0 + RR < Lw) {                                                      \
    const int t = t0 + RR;                                                 \
    const int k = bcast_i32<RR>(kv);                                       \
    if (grad && (RR % C) == 0 && t < L) ck[(t / C) * 16 + i] = f;          \
    const double fn = dot16_bcast(f, grow(s, k, i));                       \
    f = t < L ? fn : f;                                                    \
  }
        GST_FWD_STEP(0) GST_FWD_STEP(1) GST_FWD_STEP(2) GST_FWD_STEP(3)
        GST_FWD_STEP(4) GST_FWD_STEP(5) GST_FWD_STEP(6) GST_FWD_STEP(7)
        GST_FWD_STEP(8) GST_FWD_STEP(9) GST_FWD_STEP(10) GST_FWD_STEP(11)
        GST_FWD_STEP(12) GST_FWD_STEP(13) GST_FWD_STEP(14) GST_FWD_STEP(15)
#undef GST_FWD_STEP
      }
      const double p = dot16_bcast(f, reinterpret_cast<const double2*>(s.Es + i * ROW));
      double dp = 0.0;
      if (has && i < M) {
        const int64_t o = seq * M + i;
        if (R.probs) g_probs[o] = p;
        if (R.mode == MODE_LOGLIK) {
          const int32_t N = g_counts[o];
          if (N > 0) {
            if (p <= 0.0) {
              ++nonpos;
              obj = INFINITY;
            } else {
              obj -= (double)N * log(p);
              dp = -(double)N / p;
            }
          }
        } else if (R.mode == MODE_VJP) {
          dp = g_W[o];
        }
      }
      if (!grad) continue;
#define GST_DE(RR) \
  if (RR < M) dE[RR] = fma(bcast_f64<RR>(dp), f, dE[RR]);
      GST_DE(0) GST_DE(1) GST_DE(2) GST_DE(3) GST_DE(4) GST_DE(5) GST_DE(6) GST_DE(7)
      GST_DE(8) GST_DE(9) GST_DE(10) GST_DE(11) GST_DE(12) GST_DE(13) GST_DE(14) GST_DE(15)
#undef GST_DE
      const int nseg = (L + C - 1) / C;
      const int nsegw = wave_max4(nseg);
      // segment c needs its C gate indices and its checkpoint; both are
      // loaded one segment ahead of their use
      int kv_nx, kv_in;
      double ck_nx;
      {
        const int c = nsegw - 1;
        const bool seg = c >= 0 && c < nseg;
        kv_in = seg && i < C && c * C + i < L;
        kv_nx = *(kv_in ? word + c * C + i : g_gates);
        ck_nx = *(seg ? ck + c * 16 + i : ck);
        kv_nx = kv_in ? kv_nx : 0;
      }
      double b = dot16_bcast(dp, reinterpret_cast<const double2*>(s.ETs + i * ROW));
      for (int c = nsegw - 1; c >= 0; --c) {
        const bool act = c < nseg;
        const int base = c * C;
        int kv = kv_in ? kv_nx : 0;
        if (kv >= K) kv = 0;
        double fs[C];
        fs[0] = act ? ck_nx : 0.0;
        {
          const bool seg = c >= 1 && c - 1 < nseg;
          kv_in = seg && i < C && (c - 1) * C + i < L;
          kv_nx = *(kv_in ? word + (c - 1) * C + i : g_gates);
          ck_nx = *(seg ? ck + (c - 1) * 16 + i : ck);
        }
#define GST_REC(RR)                                          \
  {                                                          \
    const int k = bcast_i32<RR - 1>(kv);                     \
    fs[RR] = dot16_bcast(fs[RR - 1], grow(s, k, i));         \
  }
        GST_REC(1) GST_REC(2) GST_REC(3) GST_REC(4) GST_REC(5) GST_REC(6) GST_REC(7)
#undef GST_REC
#define GST_BWD(RR)                                          \
  {                                                          \
    const bool v = act && (base + RR < L);                   \
    const int k = bcast_i32<RR>(kv);                         \
    const int e = team * C + RR;                             \
    st_b[e * 16 + i] = b;                                    \
    st_f[e * 16 + i] = fs[RR];                               \
    if (i == 0) st_k[e] = v ? (uint8_t)k : (uint8_t)0xFF;    \
    const double bn = dot16(b, load_row(s.GTs + k * GATE_STRIDE + i * ROW)); \
    b = v ? bn : b;                                          \
  }
        GST_BWD(7) GST_BWD(6) GST_BWD(5) GST_BWD(4) GST_BWD(3) GST_BWD(2) GST_BWD(1) GST_BWD(0)
#undef GST_BWD
        wave_sync();
        flush_stash(st_b, st_f, st_k, K, acc, lane);
        wave_sync();
      }
      if (has) drho += b;
    }
    if (bad) atomicAdd(a.status + 0, (unsigned long long)bad);
    if (nonpos) {
      atomicAdd(a.status + 1, (unsigned long long)nonpos);
      atomicAdd(a.req_nonpos + T.req, (unsigned long long)nonpos);
    }
    if (grad || R.mode == MODE_LOGLIK) {
      write_slab<D>(lds_raw, obj, drho, dE, acc, M, K, R.slab + (int64_t)T.local * slab_width(D, M, K));
      staged = -1;
    }
  }
}

__global__ void queue_reset_kernel(unsigned* q, unsigned long long* req_nonpos, int n_req) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t < 6) q[16 * t] = 0u;  // the queues of the six tile groups (16 words apart)
  for (int r = t; r < n_req; r += gridDim.x * blockDim.x) req_nonpos[r] = 0ull;
}

// For every request: the sum of its tile slabs, in two stages whose order
// depends on the request's own tile count only, so that its sums are the same
// alone and in any batch.  Stage 1: block (item, c) adds the rows of chunk c
// (tiles [c R, c R + R)) over the item's 64 columns, as four interleaved
// partial sums combined in a fixed order, and stores the chunk sum over the
// chunk's first row (every read of that row is done before the barrier).
// Stage 2: the chunk sums in ascending c, the same way.  Many chunks per
// column block keep enough loads in flight to fill the chip; a single pass
// over all rows leaves a request of P columns with only P / 64 workgroups.
constexpr int RED_CHUNK = 32;

__device__ inline BatchReduceItem reduce_item(const BatchReduce& a, int b) {
  if (a.items) return a.items[b];
  BatchReduceItem it = a.one;
  it.col0 = (int64_t)b * 64;
  return it;
}

__global__ __launch_bounds__(256) void batch_reduce_chunks_kernel(const BatchReduce a) {
  __shared__ double red[4][64];
  const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
  const BatchReduceItem it = reduce_item(a, blockIdx.x);
  const int64_t x = it.col0 + tx;
  for (int c = blockIdx.y; (int64_t)c * RED_CHUNK < it.n_tiles; c += gridDim.y) {  // uniform over the block
    const int t0 = c * RED_CHUNK, t1 = min(it.n_tiles, t0 + RED_CHUNK);
    double v = 0.0;
    if (x < it.P) {
#pragma unroll
      for (int j = 0; j < RED_CHUNK / 4; ++j) {
        const int t = t0 + ty + 4 * j;
        if (t < t1) v += it.slab[(int64_t)t * it.P + x];
      }
    }
    red[ty][tx] = v;
    __syncthreads();
    if (ty == 0 && x < it.P) it.slab[(int64_t)t0 * it.P + x] = (red[0][tx] + red[1][tx]) + (red[2][tx] + red[3][tx]);
    __syncthreads();
  }
}

__global__ __launch_bounds__(256) void batch_reduce_final_kernel(const BatchReduce a) {
  __shared__ double red[4][64];
  const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
  const BatchReduceItem it = reduce_item(a, blockIdx.x);
  const int n_chunks = (it.n_tiles + RED_CHUNK - 1) / RED_CHUNK;
  const int64_t x = it.col0 + tx;
  double v = 0.0;
  if (x < it.P)
    for (int c = ty; c < n_chunks; c += 4) v += it.slab[(int64_t)c * RED_CHUNK * it.P + x];
  red[ty][tx] = v;
  __syncthreads();
  if (ty != 0 || x >= it.P) return;
  v = (red[0][tx] + red[1][tx]) + (red[2][tx] + red[3][tx]);
  const bool nonpos = a.req_nonpos[it.req] != 0;
  if (x == 0) {
    if (it.objective) *it.objective = nonpos ? INFINITY : v;
  } else if (it.grad && !nonpos) {
    it.grad[x - 1] = v;
  }
}

}  // namespace

size_t batch_lds(int kmax) { return batch_lds_bytes(kmax); }

int batch_blocks_per_cu(int D, int kmax) {
  int n = 0;
  const size_t bytes = batch_lds_bytes(kmax);
  hipError_t e = D == 16 ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, batch_kernel<16>, 256, bytes)
                         : hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, batch_kernel<4>, 256, bytes);
  return (e == hipSuccess && n > 0) ? n : 1;
}

hipError_t launch_batch(const BatchLaunch& a, int n_blocks, hipStream_t stream) {
  const size_t bytes = batch_lds_bytes(a.kmax);
  if (a.D == 16)
    gst_launch(batch_kernel<16>, dim3(n_blocks), dim3(256), bytes, stream, a);
  else if (a.D == 4)
    gst_launch(batch_kernel<4>, dim3(n_blocks), dim3(256), bytes, stream, a);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t launch_queue_reset(unsigned* q, unsigned long long* req_nonpos, int n_req, hipStream_t stream) {
  int blocks = (n_req + 255) / 256;
  if (blocks < 1) blocks = 1;
  if (blocks > 256) blocks = 256;
  gst_launch(queue_reset_kernel, dim3(blocks), dim3(256), 0, stream, q, req_nonpos, n_req);
  return hipGetLastError();
}

int batch_reduce_chunks(int64_t n_tiles) { return (int)((n_tiles + RED_CHUNK - 1) / RED_CHUNK); }

hipError_t launch_batch_reduce(const BatchReduce& a, int n_items, int max_chunks, hipStream_t stream) {
  if (n_items <= 0) return hipSuccess;
  if (max_chunks > 0)
    gst_launch(batch_reduce_chunks_kernel, dim3(n_items, max_chunks < 65535 ? max_chunks : 65535), dim3(256), 0,
               stream, a);
  gst_launch(batch_reduce_final_kernel, dim3(n_items), dim3(256), 0, stream, a);
  return hipGetLastError();
}

}  // namespace gst
