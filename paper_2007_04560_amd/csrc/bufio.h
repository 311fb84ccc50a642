// Raw buffer accesses of the Schwarz sweeps.  Every lane issues every access; a lane
// with nothing to do passes an offset past the end of the buffer, so its load returns
// zero and its store is dropped without touching memory.  With no branch around the
// accesses the hardware's count of loads in flight is the same on every path, and the
// compiler waits for exactly the loads an instruction needs.
#pragma once

#include "common.h"

namespace acch {

// Buffer resource over `bytes` bytes (raw, stride 0).
ACCH_DEV __amdgpu_buffer_rsrc_t buffer_rsrc(const void *base, unsigned bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(base), (short)0, (int)bytes, 0x00020000);
}
constexpr unsigned kPastEnd = 0x80000000u;   // offset of an idle lane's access
typedef double double_pair __attribute__((ext_vector_type(2)));
typedef float float_pair __attribute__((ext_vector_type(2)));
typedef float float_quad __attribute__((ext_vector_type(4)));
typedef unsigned word2 __attribute__((ext_vector_type(2)));
typedef unsigned word4 __attribute__((ext_vector_type(4)));

// 16 bytes at voff + soff.  (The whole loaded vector is bit-cast: taking elements of
// the builtin's result directly compiled to a narrower load.)
ACCH_DEV double2 load16(__amdgpu_buffer_rsrc_t rs, unsigned voff, unsigned soff, const double2 *) {
  const double_pair d = __builtin_bit_cast(double_pair, __builtin_amdgcn_raw_buffer_load_b128(rs, voff, soff, 0));
  return double2{d.x, d.y};
}
ACCH_DEV float4 load16(__amdgpu_buffer_rsrc_t rs, unsigned voff, unsigned soff, const float4 *) {
  const float_quad f = __builtin_bit_cast(float_quad, __builtin_amdgcn_raw_buffer_load_b128(rs, voff, soff, 0));
  return float4{f.x, f.y, f.z, f.w};
}
// one (u, v) pair of values at voff + soff
ACCH_DEV double2 load_pair(__amdgpu_buffer_rsrc_t rs, unsigned voff, unsigned soff, const double2 *) {
  return load16(rs, voff, soff, (const double2 *)nullptr);
}
ACCH_DEV float2 load_pair(__amdgpu_buffer_rsrc_t rs, unsigned voff, unsigned soff, const float2 *) {
  const float_pair f = __builtin_bit_cast(float_pair, __builtin_amdgcn_raw_buffer_load_b64(rs, voff, soff, 0));
  return float2{f.x, f.y};
}
ACCH_DEV void store_pair(__amdgpu_buffer_rsrc_t rs, unsigned voff, unsigned soff, double2 v) {
  const double_pair d{v.x, v.y};
  __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(word4, d), rs, voff, soff, 0);
}
ACCH_DEV void store_pair(__amdgpu_buffer_rsrc_t rs, unsigned voff, unsigned soff, float2 v) {
  const float_pair f{v.x, v.y};
  __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(word2, f), rs, voff, soff, 0);
}

// one value at voff + soff
ACCH_DEV double load_one(__amdgpu_buffer_rsrc_t rs, unsigned voff, unsigned soff, const double *) {
  return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(rs, voff, soff, 0));
}
ACCH_DEV float load_one(__amdgpu_buffer_rsrc_t rs, unsigned voff, unsigned soff, const float *) {
  return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(rs, voff, soff, 0));
}
ACCH_DEV unsigned load_one(__amdgpu_buffer_rsrc_t rs, unsigned voff, unsigned soff, const unsigned *) {
  return __builtin_amdgcn_raw_buffer_load_b32(rs, voff, soff, 0);
}
ACCH_DEV void store_one(__amdgpu_buffer_rsrc_t rs, unsigned voff, unsigned soff, double v) {
  __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(word2, v), rs, voff, soff, 0);
}
ACCH_DEV void store_one(__amdgpu_buffer_rsrc_t rs, unsigned voff, unsigned soff, float v) {
  __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), rs, voff, soff, 0);
}

}  // namespace acch
