// Pointwise device helpers shared by the forward and the adjoint kernels:
// periodic trilinear sampling, the data steps of Eq. (6) and batch offsets.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "kernels.h"

namespace nadmm {

// ---------------------------------------------------------------------------
// stores of results that a later kernel reads
// ---------------------------------------------------------------------------
// System scope (sc0 sc1): the L2 of the storing XCD writes them through, so
// the release at the end of the kernel finds no dirty lines to write back
// from the eight XCD caches before the next launch, whose workgroups read
// them from every XCD.  The pointers are global device memory.
//
// A VALU write to the data registers of a vector-memory store of more than
// 64 bits must come at least one wait state after the store.  The compiler
// inserts that wait for the stores it emits, not for stores inside inline
// asm, so the 128-bit form carries its own s_nop.
__device__ __forceinline__ void store_wt(float* p, float v) {
  asm volatile("global_store_dword %0, %1, off sc0 sc1" : : "v"(p), "v"(v) : "memory");
}
__device__ __forceinline__ void store_wt(float4* p, float4 v) {
  typedef float f4v __attribute__((ext_vector_type(4)));
  const f4v w = {v.x, v.y, v.z, v.w};
  asm volatile("global_store_dwordx4 %0, %1, off sc0 sc1\n\ts_nop 1" : : "v"(p), "v"(w)
               : "memory");
}
// The same at element i of a wavefront-uniform base (a scalar base plus a
// 32-bit byte offset: one array of at most 2^30 floats).
__device__ __forceinline__ void store_wt_at(float* base, uint32_t i, float4 v) {
  typedef float f4v __attribute__((ext_vector_type(4)));
  const f4v w = {v.x, v.y, v.z, v.w};
  asm volatile("global_store_dwordx4 %0, %1, %2 sc0 sc1\n\ts_nop 1" : : "v"(i << 2), "v"(w),
               "s"(base) : "memory");
}
__device__ __forceinline__ float4 ld4_at(const float* __restrict__ base, uint32_t i) {
  return *reinterpret_cast<const float4*>(reinterpret_cast<const char*>(base) + (i << 2));
}

// ---------------------------------------------------------------------------
// periodic trilinear sampling
// ---------------------------------------------------------------------------
// i mod n in [0, n) for every i; [-n, 2n) (displacements shorter than the
// grid) without a division.
__device__ __forceinline__ int wrap_index(int i, int n) {
  if (i >= -n && i < 2 * n) return i < 0 ? i + n : (i >= n ? i - n : i);
  i %= n;
  return i < 0 ? i + n : i;
}

// Grid voxel x plus displacement u, split exactly into the integer cell
// (taken modulo n) and the fraction: floor(x + u) = x + floor(u) and
// frac(x + u) = u - floor(u) since x is an integer.  Non-finite u gives a
// valid cell and a NaN fraction, never an out-of-range index.
__device__ __forceinline__ void cell(int x, float u, int n, int& i0, int& i1, float& t) {
  const float fu = floorf(u);
  t = u - fu;
  const float cl = fminf(fmaxf(fu, -1.0e9f), 1.0e9f);
  i0 = wrap_index(x + (int)cl, n);
  i1 = (i0 + 1 == n) ? 0 : i0 + 1;
}

__device__ __forceinline__ float lerpf(float a, float b, float t) { return fmaf(t, b - a, a); }

// Element offsets of the eight corners (unsigned 32-bit: a volume holds at
// most 2^30 voxels), so that loads address memory as a scalar base plus a
// 32-bit vector offset.
struct Tap {
  uint32_t o000, o100, o010, o110, o001, o101, o011, o111;
  float tx, ty, tz;
};

__device__ __forceinline__ Tap make_tap(int x, int y, int z, float ux, float uy, float uz,
                                        const Geo& g) {
  int x0, x1, y0, y1, z0, z1;
  Tap t;
  cell(x, ux, g.nx, x0, x1, t.tx);
  cell(y, uy, g.ny, y0, y1, t.ty);
  cell(z, uz, g.nz, z0, z1, t.tz);
  const uint32_t nx = g.nx, ny = g.ny;
  const uint32_t r00 = ((uint32_t)z0 * ny + y0) * nx, r01 = ((uint32_t)z0 * ny + y1) * nx;
  const uint32_t r10 = ((uint32_t)z1 * ny + y0) * nx, r11 = ((uint32_t)z1 * ny + y1) * nx;
  t.o000 = r00 + x0; t.o100 = r00 + x1;
  t.o010 = r01 + x0; t.o110 = r01 + x1;
  t.o001 = r10 + x0; t.o101 = r10 + x1;
  t.o011 = r11 + x0; t.o111 = r11 + x1;
  return t;
}

// Image element as float32: bfloat16 is the upper half of a float32.
__device__ __forceinline__ float img_at(const float* __restrict__ f, uint32_t i) {
  return *reinterpret_cast<const float*>(reinterpret_cast<const char*>(f) + (i << 2));
}
__device__ __forceinline__ float img_at(const uint16_t* __restrict__ f, uint32_t i) {
  const uint16_t b = *reinterpret_cast<const uint16_t*>(reinterpret_cast<const char*>(f) + (i << 1));
  return __uint_as_float((uint32_t)b << 16);
}

template <typename T>
__device__ __forceinline__ float sample(const T* __restrict__ f, const Tap& t) {
  const float c00 = lerpf(img_at(f, t.o000), img_at(f, t.o100), t.tx);
  const float c10 = lerpf(img_at(f, t.o010), img_at(f, t.o110), t.tx);
  const float c01 = lerpf(img_at(f, t.o001), img_at(f, t.o101), t.tx);
  const float c11 = lerpf(img_at(f, t.o011), img_at(f, t.o111), t.tx);
  return lerpf(lerpf(c00, c10, t.ty), lerpf(c01, c11, t.ty), t.tz);
}

// Two consecutive floats from a 4-byte aligned address (one 8-byte load).
typedef float float2_a4 __attribute__((ext_vector_type(2), aligned(4)));
__device__ __forceinline__ float2_a4 ld2_at(const float* __restrict__ f, uint32_t i) {
  return *reinterpret_cast<const float2_a4*>(reinterpret_cast<const char*>(f) + (i << 2));
}

// float32 fields: unless a cell of the wavefront wraps at the x edge, the
// two x taps of each corner pair are adjacent and one 8-byte load fetches
// both (half the addresses of the gather; the same values and arithmetic as
// above).  The test is wavefront-uniform.
template <>
__device__ __forceinline__ float sample(const float* __restrict__ f, const Tap& t) {
  float a000, a100, a010, a110, a001, a101, a011, a111;
  if (__all(t.o100 == t.o000 + 1)) {
    const float2_a4 p00 = ld2_at(f, t.o000), p10 = ld2_at(f, t.o010);
    const float2_a4 p01 = ld2_at(f, t.o001), p11 = ld2_at(f, t.o011);
    a000 = p00.x; a100 = p00.y; a010 = p10.x; a110 = p10.y;
    a001 = p01.x; a101 = p01.y; a011 = p11.x; a111 = p11.y;
  } else {
    a000 = img_at(f, t.o000); a100 = img_at(f, t.o100);
    a010 = img_at(f, t.o010); a110 = img_at(f, t.o110);
    a001 = img_at(f, t.o001); a101 = img_at(f, t.o101);
    a011 = img_at(f, t.o011); a111 = img_at(f, t.o111);
  }
  const float c00 = lerpf(a000, a100, t.tx);
  const float c10 = lerpf(a010, a110, t.tx);
  const float c01 = lerpf(a001, a101, t.tx);
  const float c11 = lerpf(a011, a111, t.tx);
  return lerpf(lerpf(c00, c10, t.ty), lerpf(c01, c11, t.ty), t.tz);
}

// ---------------------------------------------------------------------------
// pointwise data steps of Eq. (6) for a = w_hat - b_hat
// ---------------------------------------------------------------------------
// s = 2: v = a - J (J.a + r) / (theta + |J|^2)  (Sherman-Morrison)
// s = 1: v = a - clip(z) J / theta,  z = theta (J.a + r) / (|J|^2 + eps)
__device__ __forceinline__ void data_step(const float a[3], const float j[3], float r, float theta,
                                          float eps, int data_term, float v[3]) {
  const float ja = j[0] * a[0] + j[1] * a[1] + j[2] * a[2];
  const float jj = j[0] * j[0] + j[1] * j[1] + j[2] * j[2];
  float f;
  if (data_term == 2) {
    f = (ja + r) * __builtin_amdgcn_rcpf(theta + jj);
  } else {
    const float z = theta * (ja + r) / (jj + eps);
    f = (z / fmaxf(fabsf(z), 1.0f)) / theta;
  }
  v[0] = a[0] - j[0] * f;
  v[1] = a[1] - j[1] * f;
  v[2] = a[2] - j[2] * f;
}

// ---------------------------------------------------------------------------
// Batches: pairs of one size are stored back to back in every buffer (a
// scalar volume every V floats, a vector field every 3V, a half spectrum
// every 3 (nx/2+1) ny nz complex); the pair of a workgroup is its last grid
// index, and the kernels offset their pointers by it.
// ---------------------------------------------------------------------------
__host__ __device__ __forceinline__ size_t spectrum_elems(const Geo& g) {
  return (size_t)3 * (g.nx / 2 + 1) * g.ny * g.nz;
}
template <typename P>
__device__ __forceinline__ P* at_pair(P* p, size_t stride, int b) {
  return p ? p + stride * (size_t)b : p;
}

}  // namespace nadmm
