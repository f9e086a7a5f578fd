// Device-side helpers shared by the kernels of the one- and two-qubit path.
// Included by exactly the .hip files of this library; everything is internal.
#pragma once
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "gst_internal.h"

namespace gst {
namespace {

constexpr int TEAM = 16;               // lanes per chain
constexpr int WAVES = 4;               // waves per workgroup
constexpr int TPW = 64 / TEAM;         // chains per wave
constexpr int ROW = 18;                // padded LDS row stride in doubles
constexpr int GATE_STRIDE = 16 * ROW;  // doubles per gate matrix in LDS
constexpr int KMAX = 8;                // gates accumulated on chip
constexpr int C = 8;                   // steps per reverse segment (checkpoint interval)
constexpr int ENT = TPW * C;           // stash entries per wave (<= 64)

typedef double d4 __attribute__((ext_vector_type(4)));
typedef double d2 __attribute__((ext_vector_type(2)));

// ---------------------------------------------------------------------------
// cross-lane helpers
// ---------------------------------------------------------------------------
template <int J>
__device__ __forceinline__ int bcast_i32(int v) {
  return __builtin_amdgcn_update_dpp(0, v, 0x150 + J, 0xF, 0xF, false);
}

template <int J>
__device__ __forceinline__ double bcast_f64(double v) {
  long long x = __double_as_longlong(v);
  int lo = __builtin_amdgcn_update_dpp(0, (int)x, 0x150 + J, 0xF, 0xF, false);
  int hi = __builtin_amdgcn_update_dpp(0, (int)(x >> 32), 0x150 + J, 0xF, 0xF, false);
  return __longlong_as_double((long long)(unsigned)lo | ((long long)hi << 32));
}

// acc = fma(r[15], x@15, ... fma(r[1], x@1, fma(r[0], x@0, 0.0))) where x@j is
// x in lane j of this 16-lane row (DPP row_newbcast).  The leading s_nop
// covers the VALU-write -> DPP-read hazard on x.
__device__ __forceinline__ double dot16_bcast(double x, const double2* __restrict__ row) {
  const double2 a0 = row[0], a1 = row[1], a2 = row[2], a3 = row[3];
  const double2 a4 = row[4], a5 = row[5], a6 = row[6], a7 = row[7];
  double acc = 0.0;
  asm volatile(
      "s_nop 1\n\t"
      "v_fmac_f64_dpp %0, %1, %2 row_newbcast:0 row_mask:0xf bank_mask:0xf\n\t"
      "v_fmac_f64_dpp %0, %1, %3 row_newbcast:1 row_mask:0xf bank_mask:0xf\n\t"
      "v_fmac_f64_dpp %0, %1, %4 row_newbcast:2 row_mask:0xf bank_mask:0xf\n\t"
      "v_fmac_f64_dpp %0, %1, %5 row_newbcast:3 row_mask:0xf bank_mask:0xf\n\t"
      "v_fmac_f64_dpp %0, %1, %6 row_newbcast:4 row_mask:0xf bank_mask:0xf\n\t"
      "v_fmac_f64_dpp %0, %1, %7 row_newbcast:5 row_mask:0xf bank_mask:0xf\n\t"
      "v_fmac_f64_dpp %0, %1, %8 row_newbcast:6 row_mask:0xf bank_mask:0xf\n\t"
      "v_fmac_f64_dpp %0, %1, %9 row_newbcast:7 row_mask:0xf bank_mask:0xf\n\t"
      "v_fmac_f64_dpp %0, %1, %10 row_newbcast:8 row_mask:0xf bank_mask:0xf\n\t"
      "v_fmac_f64_dpp %0, %1, %11 row_newbcast:9 row_mask:0xf bank_mask:0xf\n\t"
      "v_fmac_f64_dpp %0, %1, %12 row_newbcast:10 row_mask:0xf bank_mask:0xf\n\t"
      "v_fmac_f64_dpp %0, %1, %13 row_newbcast:11 row_mask:0xf bank_mask:0xf\n\t"
      "v_fmac_f64_dpp %0, %1, %14 row_newbcast:12 row_mask:0xf bank_mask:0xf\n\t"
      "v_fmac_f64_dpp %0, %1, %15 row_newbcast:13 row_mask:0xf bank_mask:0xf\n\t"
      "v_fmac_f64_dpp %0, %1, %16 row_newbcast:14 row_mask:0xf bank_mask:0xf\n\t"
      "v_fmac_f64_dpp %0, %1, %17 row_newbcast:15 row_mask:0xf bank_mask:0xf"
      : "+v"(acc)
      : "v"(x), "v"(a0.x), "v"(a0.y), "v"(a1.x), "v"(a1.y), "v"(a2.x), "v"(a2.y), "v"(a3.x),
        "v"(a3.y), "v"(a4.x), "v"(a4.y), "v"(a5.x), "v"(a5.y), "v"(a6.x), "v"(a6.y), "v"(a7.x),
        "v"(a7.y));
  return acc;
}

// A 16-double row held in registers (eight 16-byte LDS reads).
struct Row16 {
  double2 a0, a1, a2, a3, a4, a5, a6, a7;
};

__device__ __forceinline__ Row16 load_row(const double* p) {
  const double2* r = reinterpret_cast<const double2*>(p);
  Row16 x;
  x.a0 = r[0];
  x.a1 = r[1];
  x.a2 = r[2];
  x.a3 = r[3];
  x.a4 = r[4];
  x.a5 = r[5];
  x.a6 = r[6];
  x.a7 = r[7];
  return x;
}

// Continues a chain: acc = fma(r[15], x@15, ... fma(r[0], x@0, acc)), the
// row already in registers.  dot16 starts from acc = 0.
__device__ __forceinline__ double dot16_from(double acc, double x, const Row16& r) {
  asm volatile(
      "s_nop 1\n\t"
      "v_fmac_f64_dpp %0, %1, %2 row_newbcast:0 row_mask:0xf bank_mask:0xf\n\t"
      "v_fmac_f64_dpp %0, %1, %3 row_newbcast:1 row_mask:0xf bank_mask:0xf\n\t"
      "v_fmac_f64_dpp %0, %1, %4 row_newbcast:2 row_mask:0xf bank_mask:0xf\n\t"
      "v_fmac_f64_dpp %0, %1, %5 row_newbcast:3 row_mask:0xf bank_mask:0xf\n\t"
      "v_fmac_f64_dpp %0, %1, %6 row_newbcast:4 row_mask:0xf bank_mask:0xf\n\t"
      "v_fmac_f64_dpp %0, %1, %7 row_newbcast:5 row_mask:0xf bank_mask:0xf\n\t"
      "v_fmac_f64_dpp %0, %1, %8 row_newbcast:6 row_mask:0xf bank_mask:0xf\n\t"
      "v_fmac_f64_dpp %0, %1, %9 row_newbcast:7 row_mask:0xf bank_mask:0xf\n\t"
      "v_fmac_f64_dpp %0, %1, %10 row_newbcast:8 row_mask:0xf bank_mask:0xf\n\t"
      "v_fmac_f64_dpp %0, %1, %11 row_newbcast:9 row_mask:0xf bank_mask:0xf\n\t"
      "v_fmac_f64_dpp %0, %1, %12 row_newbcast:10 row_mask:0xf bank_mask:0xf\n\t"
      "v_fmac_f64_dpp %0, %1, %13 row_newbcast:11 row_mask:0xf bank_mask:0xf\n\t"
      "v_fmac_f64_dpp %0, %1, %14 row_newbcast:12 row_mask:0xf bank_mask:0xf\n\t"
      "v_fmac_f64_dpp %0, %1, %15 row_newbcast:13 row_mask:0xf bank_mask:0xf\n\t"
      "v_fmac_f64_dpp %0, %1, %16 row_newbcast:14 row_mask:0xf bank_mask:0xf\n\t"
      "v_fmac_f64_dpp %0, %1, %17 row_newbcast:15 row_mask:0xf bank_mask:0xf"
      : "+v"(acc)
      : "v"(x), "v"(r.a0.x), "v"(r.a0.y), "v"(r.a1.x), "v"(r.a1.y), "v"(r.a2.x), "v"(r.a2.y), "v"(r.a3.x),
        "v"(r.a3.y), "v"(r.a4.x), "v"(r.a4.y), "v"(r.a5.x), "v"(r.a5.y), "v"(r.a6.x), "v"(r.a6.y), "v"(r.a7.x),
        "v"(r.a7.y));
  return acc;
}

// Same as dot16_bcast with the row already in registers.
__device__ __forceinline__ double dot16(double x, const Row16& r) { return dot16_from(0.0, x, r); }


__device__ __forceinline__ int uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ int64_t uniform64(int64_t v) {
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)v);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)((uint64_t)v >> 32));
  return (int64_t)(((uint64_t)hi << 32) | lo);
}

// A pointer read from memory is generic to the compiler, and a generic (flat)
// load is counted by both vmcnt and lgkmcnt, so the first LDS wait after it
// also waits for it.  This cast states that the pointer addresses global
// memory: its loads are counted by vmcnt alone and can stay in flight.
template <class T>
__device__ __forceinline__ __attribute__((address_space(1))) T* as_global(T* p) {
  return (__attribute__((address_space(1))) T*)p;
}

// 16 consecutive doubles of global memory (16-byte aligned) as a Row16.
__device__ __forceinline__ Row16 load_row_global(const double* p) {
  const auto* q = as_global(p);
  Row16 R;
  R.a0 = double2{q[0], q[1]};
  R.a1 = double2{q[2], q[3]};
  R.a2 = double2{q[4], q[5]};
  R.a3 = double2{q[6], q[7]};
  R.a4 = double2{q[8], q[9]};
  R.a5 = double2{q[10], q[11]};
  R.a6 = double2{q[12], q[13]};
  R.a7 = double2{q[14], q[15]};
  return R;
}

// max over the four 16-lane rows of a wave, as a wave-uniform value
__device__ __forceinline__ int wave_max4(int v) {
  v = max(v, __shfl_xor(v, 16));
  v = max(v, __shfl_xor(v, 32));
  return __builtin_amdgcn_readfirstlane(v);
}

// Barrier for the workgroup's LDS only: it waits for the wave's LDS accesses
// (and scalar loads), not for its global stores, which __syncthreads would
// also wait for.
__device__ __forceinline__ void lds_sync() { asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory"); }

__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// ---------------------------------------------------------------------------
// LDS layout (doubles): Gs[K][16][ROW] | GTs[K][16][ROW] | Es[16][ROW] | ETs[16][ROW] |
//   rho[16] | per wave stash: b[ENT][16], f[ENT][16] | stash gate bytes [WAVES][ENT]
// ---------------------------------------------------------------------------
struct Lds {
  double* Gs;
  double* GTs;
  double* Es;
  double* ETs;
  double* rho;
  double* stash;
  uint8_t* sk;
};

__host__ __device__ inline size_t lds_main_bytes(int K) {
  size_t d = (size_t)2 * K * GATE_STRIDE + 2 * 16 * ROW + 16 + (size_t)WAVES * 2 * ENT * 16;
  return d * 8 + (size_t)WAVES * ENT;
}

__host__ __device__ inline size_t lds_red_bytes(int K) {
  return (size_t)WAVES * (1 + 16 + 256 + (size_t)K * 256) * 8;
}

__host__ inline size_t lds_bytes(int K) {
  const size_t a = lds_main_bytes(K), b = lds_red_bytes(K);
  return a > b ? a : b;
}

__device__ __forceinline__ Lds carve(double* base, int K) {
  Lds l;
  l.Gs = base;
  l.GTs = l.Gs + (size_t)K * GATE_STRIDE;
  l.Es = l.GTs + (size_t)K * GATE_STRIDE;
  l.ETs = l.Es + 16 * ROW;
  l.rho = l.ETs + 16 * ROW;
  l.stash = l.rho + 16;
  l.sk = reinterpret_cast<uint8_t*>(l.stash + (size_t)WAVES * 2 * ENT * 16);
  return l;
}

// Parts of the gate set a kernel stages (stage_gateset's PARTS).
constexpr int STAGE_G = 1, STAGE_GT = 2, STAGE_E = 4, STAGE_ALL = 7;

// Gate set into LDS, zero-padded to 16 x 16 (and the two padding columns of
// each row zeroed): the gates (Gs), their transposes (GTs) and the effects
// with their transposes, as PARTS selects; rho always.  Workgroups of NT
// threads (64 or 256): every thread loads its entries (r, c) of every gate
// and of E up front, so the global loads are in flight together, then writes
// them.
template <int D, int NT = 256, int PARTS = STAGE_ALL>
__device__ void stage_gateset(const Lds& s, const double* __restrict__ G, const double* __restrict__ E,
                              const double* __restrict__ rho, int K, int M) {
  static_assert(NT == 64 || NT == 256, "workgroups of 64 or 256 threads");
  constexpr int U = 256 / NT;
  const int tid = threadIdx.x;
  const auto* g = as_global(G);
  const auto* e = as_global(E);
  double v[KMAX][U], ex[U];
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const int r = (tid + NT * u) >> 4, c = (tid + NT * u) & 15;
    const bool in = r < D && c < D;
#pragma unroll
    for (int k = 0; k < KMAX; ++k) {
      const bool use = k < K && in;
      const double x = g[use ? ((size_t)k * D + r) * D + c : 0];
      v[k][u] = use ? x : 0.0;
    }
    ex[u] = 0.0;
    if (PARTS & STAGE_E) {
      const bool use_e = r < M && c < D;
      const double y = e[use_e ? (size_t)r * D + c : 0];
      ex[u] = use_e ? y : 0.0;
    }
  }
  const double rh = as_global(rho)[tid < D ? tid : 0];
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const int r = (tid + NT * u) >> 4, c = (tid + NT * u) & 15;
#pragma unroll
    for (int k = 0; k < KMAX; ++k) {
      if (k < K) {
        if (PARTS & STAGE_G) {
          s.Gs[k * GATE_STRIDE + r * ROW + c] = v[k][u];
          if (c < ROW - 16) s.Gs[k * GATE_STRIDE + r * ROW + 16 + c] = 0.0;
        }
        if (PARTS & STAGE_GT) {
          s.GTs[k * GATE_STRIDE + c * ROW + r] = v[k][u];
          if (c < ROW - 16) s.GTs[k * GATE_STRIDE + r * ROW + 16 + c] = 0.0;
        }
      }
    }
    if (PARTS & STAGE_E) {
      s.Es[r * ROW + c] = ex[u];
      s.ETs[c * ROW + r] = ex[u];
      if (c < ROW - 16) {
        s.Es[r * ROW + 16 + c] = 0.0;
        s.ETs[r * ROW + 16 + c] = 0.0;
      }
    }
  }
  if (tid < 16) s.rho[tid] = tid < D ? rh : 0.0;
  __syncthreads();
}

// The same layout with one entry per thread and iteration: few registers, for
// a kernel that stages inside its hot loop and is short of them.
template <int D>
__device__ void stage_gateset_compact(const Lds& s, const double* __restrict__ G, const double* __restrict__ E,
                                      const double* __restrict__ rho, int K, int M) {
  const int tid = threadIdx.x;
  for (int x = tid; x < K * 16 * ROW; x += blockDim.x) {
    const int k = x / (16 * ROW), r = (x / ROW) % 16, c = x % ROW;
    double g = 0.0, gt = 0.0;
    if (r < D && c < D) {
      g = G[((size_t)k * D + r) * D + c];
      gt = G[((size_t)k * D + c) * D + r];
    }
    s.Gs[x] = g;
    s.GTs[x] = gt;
  }
  for (int x = tid; x < 16 * ROW; x += blockDim.x) {
    const int r = x / ROW, c = x % ROW;
    s.Es[x] = (r < M && c < D) ? E[(size_t)r * D + c] : 0.0;
    s.ETs[x] = (c < M && r < D) ? E[(size_t)c * D + r] : 0.0;
  }
  if (tid < 16) s.rho[tid] = tid < D ? rho[tid] : 0.0;
  __syncthreads();
}

__device__ __forceinline__ const double2* grow(const Lds& s, int k, int i) {
  return reinterpret_cast<const double2*>(s.Gs + k * GATE_STRIDE + i * ROW);
}
__device__ __forceinline__ const double2* gtrow(const Lds& s, int k, int i) {
  return reinterpret_cast<const double2*>(s.GTs + k * GATE_STRIDE + i * ROW);
}

// dG_k += sum over the wave's stashed steps with gate k of b f^T, four steps
// per MFMA 16x16x4 (A[i][z] = b_z[i], B[z][j] = f_z[j]).
__device__ __forceinline__ void flush_stash(const double* st_b, const double* st_f, const uint8_t* st_k, int K,
                                            d4 (&acc)[KMAX], int lane) {
  const int i = lane & 15;
  const int my_k = lane < ENT ? (int)st_k[lane] : 0xFF;
#pragma unroll
  for (int k = 0; k < KMAX; ++k) {
    if (k < K) {
      unsigned long long mask = __ballot(my_k == k);
      while (mask) {
        int e4[4];
#pragma unroll
        for (int z = 0; z < 4; ++z) {
          if (mask) {
            e4[z] = __ffsll((long long)mask) - 1;
            mask &= mask - 1;
          } else {
            e4[z] = -1;
          }
        }
        const int sel = lane >> 4;
        const int e = sel == 0 ? e4[0] : sel == 1 ? e4[1] : sel == 2 ? e4[2] : e4[3];
        const double av = e >= 0 ? st_b[e * 16 + i] : 0.0;
        const double bv = e >= 0 ? st_f[e * 16 + i] : 0.0;
        acc[k] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc[k], 0, 0, 0);
      }
    }
  }
}

// Adds the four chains of each wave and the four waves and writes the slab
// row `slab` = [objective | drho (D) | dE (M*D) | dG (K*D*D)] (the caller
// picks the row).  Reuses the LDS from its start: the staged gate set is
// overwritten.
template <int D>
__device__ void write_slab(double* lds_raw, double obj, double drho, double (&dE)[16], d4 (&acc)[KMAX], int M,
                           int K, double* slab) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  __syncthreads();  // LDS is reused from here on
  const int P16 = 1 + 16 + 256 + K * 256;
  double* mine = lds_raw + (size_t)wave * P16;
  double o = obj;
#pragma unroll
  for (int sh = 1; sh < 64; sh <<= 1) o += __shfl_xor(o, sh);
  double dr = drho;
  dr += __shfl_xor(dr, 16);
  dr += __shfl_xor(dr, 32);
#pragma unroll
  for (int m = 0; m < 16; ++m) {
    dE[m] += __shfl_xor(dE[m], 16);
    dE[m] += __shfl_xor(dE[m], 32);
  }
  if (lane == 0) mine[0] = o;
  if (lane < 16) {
    mine[1 + lane] = dr;
#pragma unroll
    for (int m = 0; m < 16; ++m) mine[17 + m * 16 + lane] = dE[m];
  }
  // tile element C[r][c] sits in lane 16*(r&3)+c, register r>>2
#pragma unroll
  for (int k = 0; k < KMAX; ++k) {
    if (k < K) {
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int r = 4 * v + (lane >> 4), c = lane & 15;
        mine[273 + k * 256 + r * 16 + c] = acc[k][v];
      }
    }
  }
  __syncthreads();
  const int64_t P = slab_width(D, M, K);
  double* out = slab;
  const double* red = lds_raw;
  for (int x = tid; x < P; x += blockDim.x) {
    int src;
    if (x == 0) {
      src = 0;
    } else if (x < 1 + D) {
      src = x;
    } else if (x < 1 + D + M * D) {
      const int y = x - 1 - D;
      src = 17 + (y / D) * 16 + (y % D);
    } else {
      const int y = x - 1 - D - M * D;
      const int k = y / (D * D), r = (y / D) % D, c = y % D;
      src = 273 + k * 256 + r * 16 + c;
    }
    double v = red[src];
    v += red[P16 + src];
    v += red[2 * P16 + src];
    v += red[3 * P16 + src];
    out[x] = v;
  }
}

// C = A B for 16 x 16 matrices in the gate layout (LDS), by one wave on the
// FP64 matrix cores: four 16x16x4 MFMAs, the k-th (k = 0..3) adding columns
// 4k..4k+3 of A times rows 4k..4k+3 of B.  Lane l supplies A[l & 15][4k + (l >> 4)]
// and B[4k + (l >> 4)][l & 15] and ends with C[4v + (l >> 4)][l & 15] in
// register v.  Each MFMA adds its four products as sequential fused
// multiply-adds in ascending order, so every entry is the same fused
// multiply-add chain over j = 0..15 as a dot product with a zero start.
__device__ __forceinline__ void wave_matmul(double* C, const double* A, const double* B, int lane) {
  const int i = lane & 15, t = lane >> 4;
  double a[4], b[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    a[k] = A[i * ROW + 4 * k + t];
    b[k] = B[(4 * k + t) * ROW + i];
  }
  d4 acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int k = 0; k < 4; ++k) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a[k], b[k], acc, 0, 0, 0);
#pragma unroll
  for (int v = 0; v < 4; ++v) C[(4 * v + t) * ROW + i] = acc[v];
  wave_sync();
}

// The trunk's jump matrices into the wave's slots js[e * GATE_STRIDE]: slot 0
// = G_{g_per-1} ... G_{g_0} of the pattern (reverse: its transpose G_{g_0}^T
// ... G_{g_per-1}^T, from the transposed gate set), slot e = slot e-1 squared.
__device__ inline void build_jumps(double* js, const double* gates, uint32_t pat, int g3, int levels, bool rev,
                            int lane) {
  const int per = (int)(pat & 0xffu);
  const int g[4] = {(int)((pat >> 8) & 0xffu), (int)((pat >> 16) & 0xffu), (int)((pat >> 24) & 0xffu), g3};
  const int i = lane & 15, t = lane >> 4;
  if (per == 1) {
#pragma unroll
    for (int u = 0; u < 4; ++u) js[i * ROW + 4 * u + t] = gates[g[0] * GATE_STRIDE + i * ROW + 4 * u + t];
    wave_sync();
  } else {
    const double* src = gates + g[rev ? per - 1 : 0] * GATE_STRIDE;
    for (int k = 1; k < per; ++k) {  // the last product lands in slot 0
      double* dst = js + (((per - 1 - k) & 1) ? GATE_STRIDE : 0);
      wave_matmul(dst, gates + g[rev ? per - 1 - k : k] * GATE_STRIDE, src, lane);
      src = dst;
    }
  }
  for (int e = 1; e < levels; ++e)
    wave_matmul(js + e * GATE_STRIDE, js + (e - 1) * GATE_STRIDE, js + (e - 1) * GATE_STRIDE, lane);
}

}  // namespace

// Slab sums in two deterministic stages.  Stage 1: block (x, g) adds slabs
// [g*per, (g+1)*per) for 64 consecutive entries, four interleaved partial
// sums combined in a fixed order.  Stage 2: entry p adds the stage-1
// partials in ascending g, plus an optional extra vector on the rho entries.
__device__ __forceinline__ void slab_sum_stage1(const double* __restrict__ slab, int n_slabs, int64_t P, int per,
                                                double* __restrict__ part, int64_t bx, int g) {
  __shared__ double red[4][64];
  const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
  const int64_t p = bx * 64 + tx;
  const int w0 = g * per, w1 = min(n_slabs, w0 + per);
  double v = 0.0;
  if (p < P)
    for (int w = w0 + ty; w < w1; w += 4) v += slab[(int64_t)w * P + p];
  red[ty][tx] = v;
  __syncthreads();
  if (ty == 0 && p < P) part[(int64_t)g * P + p] = (red[0][tx] + red[1][tx]) + (red[2][tx] + red[3][tx]);
}

__device__ __forceinline__ void slab_sum_stage2(const double* __restrict__ part, int n_part, int64_t P,
                                                double* objective, double* grad, const double* __restrict__ extra_rho,
                                                int D, int64_t bx) {
  // An objective partial of +inf marks p <= 0 with N > 0 in this evaluation:
  // the objective is then +inf and the gradient is not written.  Every block
  // checks the n_part (<= 64) objective partials itself.
  __shared__ double red[4][64];
  __shared__ int nonpos_sh;
  const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
  const int64_t x = bx * 64 + tx;
  double v = 0.0;
  if (x < P)
    for (int g = ty; g < n_part; g += 4) v += part[(int64_t)g * P + x];
  red[ty][tx] = v;
  if (ty == 1) {
    const bool inf = tx < n_part && isinf(part[(int64_t)tx * P]);
    const bool any = __ballot(inf) != 0ull;
    if (tx == 0) nonpos_sh = any ? 1 : 0;
  }
  __syncthreads();
  const bool nonpos = nonpos_sh != 0;
  if (ty != 0 || x >= P) return;
  v = (red[0][tx] + red[1][tx]) + (red[2][tx] + red[3][tx]);
  if (extra_rho && x >= 1 && x <= D) v += extra_rho[x - 1];
  if (x == 0) {
    if (objective) *objective = nonpos ? INFINITY : v;
  } else if (grad && !nonpos) {
    grad[x - 1] = v;
  }
}

}  // namespace gst
