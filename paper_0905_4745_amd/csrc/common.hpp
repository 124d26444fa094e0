// Shared device-side helpers: scalar/complex value types, arithmetic and
// workgroup reductions.  gfx950 wavefronts are 64 lanes wide.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mn {

constexpr int kWave = 64;

struct cf {  // complex float, interleaved
  float re, im;
};
struct alignas(16) cd {  // complex double, interleaved
  double re, im;
};

// ---- type traits ----------------------------------------------------------
template <typename V> struct VT;
template <> struct VT<double> { using real = double; static constexpr bool cplx = false; using wide = double; };
template <> struct VT<float> { using real = float; static constexpr bool cplx = false; using wide = double; };
template <> struct VT<cd> { using real = double; static constexpr bool cplx = true; using wide = cd; };
template <> struct VT<cf> { using real = float; static constexpr bool cplx = true; using wide = cd; };

// ---- construction / conversion -------------------------------------------
template <typename V> __host__ __device__ inline V vzero();
template <> __host__ __device__ inline double vzero<double>() { return 0.0; }
template <> __host__ __device__ inline float vzero<float>() { return 0.0f; }
template <> __host__ __device__ inline cd vzero<cd>() { return cd{0.0, 0.0}; }
template <> __host__ __device__ inline cf vzero<cf>() { return cf{0.0f, 0.0f}; }

template <typename V> __host__ __device__ inline V vmake(double re, double im);
template <> __host__ __device__ inline double vmake<double>(double re, double) { return re; }
template <> __host__ __device__ inline float vmake<float>(double re, double) { return (float)re; }
template <> __host__ __device__ inline cd vmake<cd>(double re, double im) { return cd{re, im}; }
template <> __host__ __device__ inline cf vmake<cf>(double re, double im) { return cf{(float)re, (float)im}; }

__host__ __device__ inline double vre(double a) { return a; }
__host__ __device__ inline float vre(float a) { return a; }
__host__ __device__ inline double vre(cd a) { return a.re; }
__host__ __device__ inline float vre(cf a) { return a.re; }
__host__ __device__ inline double vim(double) { return 0.0; }
__host__ __device__ inline float vim(float) { return 0.0f; }
__host__ __device__ inline double vim(cd a) { return a.im; }
__host__ __device__ inline float vim(cf a) { return a.im; }

// convert between precisions of the same kind (complex <-> complex, real <-> real)
template <typename To, typename From> __host__ __device__ inline To vconv(From a) {
  return vmake<To>((double)vre(a), (double)vim(a));
}

// ---- arithmetic -----------------------------------------------------------
__host__ __device__ inline double vconj(double a) { return a; }
__host__ __device__ inline float vconj(float a) { return a; }
__host__ __device__ inline cd vconj(cd a) { return cd{a.re, -a.im}; }
__host__ __device__ inline cf vconj(cf a) { return cf{a.re, -a.im}; }

__host__ __device__ inline double vadd(double a, double b) { return a + b; }
__host__ __device__ inline float vadd(float a, float b) { return a + b; }
__host__ __device__ inline cd vadd(cd a, cd b) { return cd{a.re + b.re, a.im + b.im}; }
__host__ __device__ inline cf vadd(cf a, cf b) { return cf{a.re + b.re, a.im + b.im}; }

__host__ __device__ inline double vsub(double a, double b) { return a - b; }
__host__ __device__ inline float vsub(float a, float b) { return a - b; }
__host__ __device__ inline cd vsub(cd a, cd b) { return cd{a.re - b.re, a.im - b.im}; }
__host__ __device__ inline cf vsub(cf a, cf b) { return cf{a.re - b.re, a.im - b.im}; }

__host__ __device__ inline double vmul(double a, double b) { return a * b; }
__host__ __device__ inline float vmul(float a, float b) { return a * b; }
__host__ __device__ inline cd vmul(cd a, cd b) {
  return cd{a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
__host__ __device__ inline cf vmul(cf a, cf b) {
  return cf{a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
// conj(a) * b
__host__ __device__ inline double vcmul(double a, double b) { return a * b; }
__host__ __device__ inline float vcmul(float a, float b) { return a * b; }
__host__ __device__ inline cd vcmul(cd a, cd b) {
  return cd{a.re * b.re + a.im * b.im, a.re * b.im - a.im * b.re};
}
__host__ __device__ inline cf vcmul(cf a, cf b) {
  return cf{a.re * b.re + a.im * b.im, a.re * b.im - a.im * b.re};
}
// acc + a * b
__host__ __device__ inline double vfma(double a, double b, double c) { return fma(a, b, c); }
__host__ __device__ inline float vfma(float a, float b, float c) { return fmaf(a, b, c); }
__host__ __device__ inline cd vfma(cd a, cd b, cd c) {
  return cd{fma(a.re, b.re, fma(-a.im, b.im, c.re)), fma(a.re, b.im, fma(a.im, b.re, c.im))};
}
__host__ __device__ inline cf vfma(cf a, cf b, cf c) {
  return cf{fmaf(a.re, b.re, fmaf(-a.im, b.im, c.re)), fmaf(a.re, b.im, fmaf(a.im, b.re, c.im))};
}
// acc + conj(a) * b
__host__ __device__ inline double vcfma(double a, double b, double c) { return fma(a, b, c); }
__host__ __device__ inline float vcfma(float a, float b, float c) { return fmaf(a, b, c); }
__host__ __device__ inline cd vcfma(cd a, cd b, cd c) {
  return cd{fma(a.re, b.re, fma(a.im, b.im, c.re)), fma(a.re, b.im, fma(-a.im, b.re, c.im))};
}
__host__ __device__ inline cf vcfma(cf a, cf b, cf c) {
  return cf{fmaf(a.re, b.re, fmaf(a.im, b.im, c.re)), fmaf(a.re, b.im, fmaf(-a.im, b.re, c.im))};
}
__host__ __device__ inline double vscale(double a, double s) { return a * s; }
__host__ __device__ inline float vscale(float a, float s) { return a * s; }
__host__ __device__ inline cd vscale(cd a, double s) { return cd{a.re * s, a.im * s}; }
__host__ __device__ inline cf vscale(cf a, float s) { return cf{a.re * s, a.im * s}; }

__host__ __device__ inline double vabs2(double a) { return a * a; }
__host__ __device__ inline float vabs2(float a) { return a * a; }
__host__ __device__ inline double vabs2(cd a) { return a.re * a.re + a.im * a.im; }
__host__ __device__ inline float vabs2(cf a) { return a.re * a.re + a.im * a.im; }

__host__ __device__ inline bool vfinite(double a) { return isfinite(a); }
__host__ __device__ inline bool vfinite(float a) { return isfinite(a); }
__host__ __device__ inline bool vfinite(cd a) { return isfinite(a.re) && isfinite(a.im); }
__host__ __device__ inline bool vfinite(cf a) { return isfinite(a.re) && isfinite(a.im); }

// multiply by -i (used in radix-4 butterflies); real types never call it
__device__ inline cd vmul_negi(cd a) { return cd{a.im, -a.re}; }
__device__ inline cf vmul_negi(cf a) { return cf{a.im, -a.re}; }

// ---- DPP lane exchanges (VALU, no LDS traffic) ------------------------------
// quad_perm xor 1, quad_perm xor 2, mirror within 8 lanes, mirror within 16,
// rotation by 8 within 16.
constexpr int kDppXor1 = 0xB1, kDppXor2 = 0x4E, kDppHalfMirror = 0x141, kDppMirror = 0x140;
constexpr int kDppRor8 = 0x128;  // rotate right by 8 within 16-lane rows (= lane ^ 8)
template <int CTRL> __device__ inline int dpp_i(int v) {
  return __builtin_amdgcn_update_dpp(0, v, CTRL, 0xF, 0xF, false);
}
template <int CTRL> __device__ inline float dpp(float v) { return __int_as_float(dpp_i<CTRL>(__float_as_int(v))); }
template <int CTRL> __device__ inline double dpp(double v) {
  const int lo = dpp_i<CTRL>(__double2loint(v)), hi = dpp_i<CTRL>(__double2hiint(v));
  return __hiloint2double(hi, lo);
}
template <int CTRL> __device__ inline cd dpp(cd v) { return cd{dpp<CTRL>(v.re), dpp<CTRL>(v.im)}; }
template <int CTRL> __device__ inline cf dpp(cf v) { return cf{dpp<CTRL>(v.re), dpp<CTRL>(v.im)}; }

// Sum over aligned groups of 8 (16) consecutive lanes; every lane of the
// group receives the sum.  The combination order is fixed.
template <typename S> __device__ inline S sum8(S v) {
  v = vadd(v, dpp<kDppXor1>(v));
  v = vadd(v, dpp<kDppXor2>(v));
  v = vadd(v, dpp<kDppHalfMirror>(v));
  return v;
}
template <typename S> __device__ inline S sum16(S v) { return vadd(sum8(v), dpp<kDppMirror>(sum8(v))); }

// ---- wave / workgroup reductions (fixed order: deterministic) -------------
// Sum over the 64-lane wave: DPP within 16-lane rows, then two shuffles.
__device__ inline double wave_sum(double v) {
  v = sum16(v);
  v += __shfl_xor(v, 16, kWave);
  v += __shfl_xor(v, 32, kWave);
  return v;
}
__device__ inline float wave_sum(float v) {
  v = sum16(v);
  v += __shfl_xor(v, 16, kWave);
  v += __shfl_xor(v, 32, kWave);
  return v;
}
__device__ inline cd wave_sum(cd v) { return cd{wave_sum(v.re), wave_sum(v.im)}; }
__device__ inline cf wave_sum(cf v) { return cf{wave_sum(v.re), wave_sum(v.im)}; }
__device__ inline double wave_max(double v) {
#pragma unroll
  for (int off = kWave / 2; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, kWave));
  return v;
}

// Sum over the workgroup; every thread gets the result.  `red` must hold
// blockDim.x / 64 entries.  Contains two barriers.
template <typename S>
__device__ inline S block_sum(S v, S* red) {
  const int lane = threadIdx.x & (kWave - 1);
  const int w = threadIdx.x / kWave;
  const int nw = blockDim.x / kWave;
  v = wave_sum(v);
  __syncthreads();
  if (lane == 0) red[w] = v;
  __syncthreads();
  S t = red[0];
  for (int i = 1; i < nw; ++i) t = vadd(t, red[i]);
  return t;
}

__device__ inline double block_max(double v, double* red) {
  const int lane = threadIdx.x & (kWave - 1);
  const int w = threadIdx.x / kWave;
  const int nw = blockDim.x / kWave;
  v = wave_max(v);
  __syncthreads();
  if (lane == 0) red[w] = v;
  __syncthreads();
  double t = red[0];
  for (int i = 1; i < nw; ++i) t = fmax(t, red[i]);
  return t;
}

__host__ __device__ inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

// Block coordinates of a kernel body: the hardware ones for a plain launch,
// or a system's own grid inside a batched launch (kernels.hpp, BGrid).
struct Bk {
  int x, y, z;
  int gx, gy, gz;
};
__device__ inline Bk bk_hw() {
  return Bk{(int)blockIdx.x, (int)blockIdx.y, (int)blockIdx.z, (int)gridDim.x, (int)gridDim.y, (int)gridDim.z};
}


}  // namespace mn
