// Device-side building blocks shared by the PT-TEBD kernels (gfx950).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ptt {

// ---------------------------------------------------------------- complex
template <typename T> struct cvec;
template <> struct cvec<double> { using type = double2; };
template <> struct cvec<float> { using type = float2; };
template <typename T> using cx = typename cvec<T>::type;

template <typename T> __host__ __device__ inline cx<T> mk(T re, T im) { cx<T> z; z.x = re; z.y = im; return z; }
template <typename T> __device__ inline cx<T> cadd(cx<T> a, cx<T> b) { return mk<T>(a.x + b.x, a.y + b.y); }
template <typename T> __device__ inline cx<T> csub(cx<T> a, cx<T> b) { return mk<T>(a.x - b.x, a.y - b.y); }
template <typename T> __device__ inline cx<T> cmul(cx<T> a, cx<T> b) {
  return mk<T>(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
template <typename T> __device__ inline cx<T> cconj(cx<T> a) { return mk<T>(a.x, -a.y); }
template <typename T> __device__ inline cx<T> cscale(cx<T> a, T s) { return mk<T>(a.x * s, a.y * s); }
// acc += a * b
template <typename T> __device__ inline void cfma(cx<T>& acc, cx<T> a, cx<T> b) {
  acc.x = fma(a.x, b.x, acc.x);
  acc.x = fma(-a.y, b.y, acc.x);
  acc.y = fma(a.x, b.y, acc.y);
  acc.y = fma(a.y, b.x, acc.y);
}
// acc += conj(a) * b
template <typename T> __device__ inline void cfmaconj(cx<T>& acc, cx<T> a, cx<T> b) {
  acc.x = fma(a.x, b.x, acc.x);
  acc.x = fma(a.y, b.y, acc.x);
  acc.y = fma(a.x, b.y, acc.y);
  acc.y = fma(-a.y, b.x, acc.y);
}
template <typename T> __device__ inline T cabs2(cx<T> a) { return a.x * a.x + a.y * a.y; }

// ------------------------------------------------------------ reductions
__device__ inline double warp_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Sum over a fully active wave by DPP lane moves (quad permutations, row
// rotations, row broadcasts): register-to-register, no LDS round trip.  The
// total is read from lane 63 and returned to every lane.
template <int CTRL, int ROW_MASK> __device__ inline double dpp_move(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)b, CTRL, ROW_MASK, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, ROW_MASK, 0xf, false);
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}
__device__ inline double wave_sum_dpp(double v) {
  v += dpp_move<0xB1, 0xF>(v);    // quad_perm [1,0,3,2]
  v += dpp_move<0x4E, 0xF>(v);    // quad_perm [2,3,0,1]: every lane holds its quad's sum
  v += dpp_move<0x124, 0xF>(v);   // row_ror 4
  v += dpp_move<0x128, 0xF>(v);   // row_ror 8: every lane holds its row's sum
  v += dpp_move<0x142, 0xA>(v);   // row_bcast 15 into rows 1 and 3
  v += dpp_move<0x143, 0xC>(v);   // row_bcast 31 into rows 2 and 3: lane 63 holds the total
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)b, 63), hi = __builtin_amdgcn_readlane((int)(b >> 32), 63);
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

// Sum over each half of a fully active wave (lanes 0-31, 32-63) by DPP
// moves; the half's total is valid in its last lane (31 or 63).
__device__ inline double half_wave_sum_dpp(double v) {
  v += dpp_move<0xB1, 0xF>(v);    // quad_perm [1,0,3,2]
  v += dpp_move<0x4E, 0xF>(v);    // quad_perm [2,3,0,1]
  v += dpp_move<0x124, 0xF>(v);   // row_ror 4
  v += dpp_move<0x128, 0xF>(v);   // row_ror 8: every lane holds its row's sum
  v += dpp_move<0x142, 0xA>(v);   // row_bcast 15 into rows 1 and 3
  return v;
}

// Loads and stores through pointers known to be in global memory.  A
// pointer read from a job descriptor has no address space for the compiler,
// which then emits flat instructions; those count against the LDS counter as
// well, so every LDS wait (and every barrier) also waits for them.
#define PTT_GLOBAL __attribute__((address_space(1)))
typedef double ptt_d2v __attribute__((ext_vector_type(2)));
__device__ inline double2 gload(const double2* p) {
  const ptt_d2v v = *(const PTT_GLOBAL ptt_d2v*)p;
  return make_double2(v.x, v.y);
}
__device__ inline void gstore(double2* p, double2 v) {
  ptt_d2v t;
  t.x = v.x;
  t.y = v.y;
  *(PTT_GLOBAL ptt_d2v*)p = t;
}
__device__ inline void gstore(double* p, double v) { *(PTT_GLOBAL double*)p = v; }
__device__ inline double gload(const double* p) { return *(const PTT_GLOBAL double*)p; }

// Block-wide sum of one double (all threads get the result).  `red` must
// hold one double per wave.
__device__ inline double block_sum(double v, double* red) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int nw = (blockDim.x + 63) >> 6;
  v = warp_sum(v);
  __syncthreads();
  if (lane == 0) red[wid] = v;
  __syncthreads();
  double s = 0.0;
  for (int i = 0; i < nw; ++i) s += red[i];
  return s;
}

// block_sum with DPP wave sums (no LDS round trips inside a wave).  `red`
// must hold one double per wave.
__device__ inline double block_sum_dpp(double v, double* red) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int nw = (blockDim.x + 63) >> 6;
  v = wave_sum_dpp(v);
  __syncthreads();
  if (lane == 0) red[wid] = v;
  __syncthreads();
  return wave_sum_dpp(lane < nw ? red[lane] : 0.0);
}

// ------------------------------------------------------------------ RNG
// SplitMix64 finaliser (Steele, Lea, Flood 2014) used as a counter-based
// generator: value = mix(seed + counter * golden_gamma).
__host__ __device__ inline uint64_t splitmix64(uint64_t x) {
  x += 0x9E3779B97F4A7C15ull;
  x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
  x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
  return x ^ (x >> 31);
}
__device__ inline double u01(uint64_t bits) { return ((bits >> 11) + 0.5) * (1.0 / 9007199254740992.0); }

}  // namespace ptt
