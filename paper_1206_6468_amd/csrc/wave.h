// Wavefront-level helpers shared by the kernels: DPP reductions over the 64 lanes
// of a wavefront (plain and compensated) and global-address-space pointer types.
#pragma once
#include <hip/hip_runtime.h>

#include "special.h"

namespace nfhmm {

// Wavefront reductions with DPP lane moves: within quads, half-rows and rows of
// 16, then across rows with the row broadcasts; the total lands in lane 63 and
// is read back to every lane.
template <int CTRL, int ROWS>
__device__ __forceinline__ float dpp_mov(float old, float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(__float_as_int(old), __float_as_int(v), CTRL, ROWS, 0xf, false));
}
__device__ __forceinline__ float lane63(float v) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 63));
}
// Global-memory pointers (address space 1), so that loads and stores are
// global_* instructions, which count only against vmcnt.  A kernel copies the
// descriptor fields it needs into such locals before its first store: loaded
// then, they are scalar loads kept in SGPRs; read after a store, the compiler
// must reload them per lane (the store might have changed the descriptor).
typedef float vf2 __attribute__((ext_vector_type(2)));
typedef float vf4 __attribute__((ext_vector_type(4)));
typedef unsigned int vu2 __attribute__((ext_vector_type(2)));
typedef __attribute__((address_space(1))) float gfloat;
typedef __attribute__((address_space(1))) vf2 gfloat2;
typedef __attribute__((address_space(1))) vf4 gfloat4;
typedef __attribute__((address_space(1))) vu2 guint2;
typedef __attribute__((address_space(1))) uint16_t gu16;
__device__ __forceinline__ gfloat *gptr(float *p) { return (gfloat *)p; }
__device__ __forceinline__ const gfloat *gptr(const float *p) { return (const gfloat *)p; }
__device__ __forceinline__ gfloat2 *gptr(float2 *p) { return (gfloat2 *)p; }
__device__ __forceinline__ const gfloat2 *gptr(const float2 *p) { return (const gfloat2 *)p; }
__device__ __forceinline__ gu16 *gptr(uint16_t *p) { return (gu16 *)p; }
__device__ __forceinline__ const gu16 *gptr(const uint16_t *p) { return (const gu16 *)p; }

__device__ __forceinline__ float wave_sum(float x) {
  x += dpp_mov<0xb1, 0xf>(0.0f, x);      // quad_perm [1,0,3,2]
  x += dpp_mov<0x4e, 0xf>(0.0f, x);      // quad_perm [2,3,0,1]
  x += dpp_mov<0x141, 0xf>(0.0f, x);     // row_half_mirror
  x += dpp_mov<0x140, 0xf>(0.0f, x);     // row_mirror
  x += dpp_mov<0x142, 0xa>(0.0f, x);     // row_bcast:15 into rows 1, 3
  x += dpp_mov<0x143, 0xc>(0.0f, x);     // row_bcast:31 into rows 2, 3
  return lane63(x);
}
__device__ __forceinline__ float wave_max(float x) {
  const float ninf = -INFINITY;
  x = fmaxf(x, dpp_mov<0xb1, 0xf>(ninf, x));
  x = fmaxf(x, dpp_mov<0x4e, 0xf>(ninf, x));
  x = fmaxf(x, dpp_mov<0x141, 0xf>(ninf, x));
  x = fmaxf(x, dpp_mov<0x140, 0xf>(ninf, x));
  x = fmaxf(x, dpp_mov<0x142, 0xa>(ninf, x));
  x = fmaxf(x, dpp_mov<0x143, 0xc>(ninf, x));
  return lane63(x);
}
__device__ __forceinline__ Comp comp_dpp_step(Comp c, Comp d) { return comp_merge(c, d); }
template <int CTRL, int ROWS>
__device__ __forceinline__ Comp comp_mov(Comp c) {
  Comp d;
  d.hi = dpp_mov<CTRL, ROWS>(0.0f, c.hi);
  d.lo = dpp_mov<CTRL, ROWS>(0.0f, c.lo);
  return d;
}
__device__ __forceinline__ Comp wave_comp(Comp c) {
  c = comp_merge(c, comp_mov<0xb1, 0xf>(c));
  c = comp_merge(c, comp_mov<0x4e, 0xf>(c));
  c = comp_merge(c, comp_mov<0x141, 0xf>(c));
  c = comp_merge(c, comp_mov<0x140, 0xf>(c));
  c = comp_merge(c, comp_mov<0x142, 0xa>(c));
  c = comp_merge(c, comp_mov<0x143, 0xc>(c));
  Comp r;
  r.hi = lane63(c.hi);
  r.lo = lane63(c.lo);
  return r;
}

}  // namespace nfhmm
