// Kernel instances for one value of NT = n_pad / 16, selected at build time
// with -DHOPF_NT=<k>; the build compiles this file once per NT.
#include "hopf_device.h"

#ifndef HOPF_NT
#error "HOPF_NT must be defined"
#endif

#define HOPF_CAT2(a, b) a##b
#define HOPF_CAT(a, b) HOPF_CAT2(a, b)

namespace hopf {

// number of control components held in registers (the system's m is rounded up)
static const int kMM[] = {1, 2, 3, 4, 5, 6, 8, 10, 12, 16};

// waves: 4, or 8 for the FP32 kernel (the node blocks of a tile over twice
// as many waves, for launches with few tiles)
pdhg_fn HOPF_CAT(pdhg_lookup_nt, HOPF_NT)(int m, int prec, int waves, int *MM_out) {
#if HOPF_NT > 8
  (void)m; (void)prec; (void)waves;
  if (MM_out) *MM_out = 0;
  return nullptr;
#else
  int MM = 0;
  for (int v : kMM)
    if (v >= m) { MM = v; break; }
  if (MM_out) *MM_out = MM;
  if (prec == HOPF_FP64) {
#if HOPF_NT <= 2
    if (waves != WAVES) return nullptr;
    switch (MM) {
      case 1: return k_pdhg<double, HOPF_NT, 1, WAVES>;
      case 2: return k_pdhg<double, HOPF_NT, 2, WAVES>;
      case 3: return k_pdhg<double, HOPF_NT, 3, WAVES>;
      case 4: return k_pdhg<double, HOPF_NT, 4, WAVES>;
      default: return nullptr;
    }
#else
    return nullptr;
#endif
  }
#define HOPF_F32(MMV)                                                           \
  case MMV:                                                                     \
    return waves == 8 ? k_pdhg<float, HOPF_NT, MMV, 8> : k_pdhg<float, HOPF_NT, MMV, WAVES>;
  if (waves != WAVES && waves != 8) return nullptr;
  switch (MM) {
    HOPF_F32(1)
    HOPF_F32(2)
    HOPF_F32(3)
    HOPF_F32(4)
    HOPF_F32(5)
    HOPF_F32(6)
    HOPF_F32(8)
    HOPF_F32(10)
    HOPF_F32(12)
    HOPF_F32(16)
    default: return nullptr;
  }
#undef HOPF_F32
#endif
}

pdhg_fn HOPF_CAT(wide_lookup_nt, HOPF_NT)(int m) {
#if HOPF_NT > 8
  (void)m;
  return nullptr;
#else
  int MM = 0;
  for (int v : kMM)
    if (v >= m) { MM = v; break; }
  // one node block of the table in LDS, two workgroups per compute unit
  if ((size_t)NODE_BLOCK * MM * wide_row_stride(HOPF_NT) * 4 > 76 * 1024) return nullptr;
  switch (MM) {
    case 1: return k_pdhg_wide<HOPF_NT, 1>;
    case 2: return k_pdhg_wide<HOPF_NT, 2>;
    case 3: return k_pdhg_wide<HOPF_NT, 3>;
    case 4: return k_pdhg_wide<HOPF_NT, 4>;
    case 5: return k_pdhg_wide<HOPF_NT, 5>;
    case 6: return k_pdhg_wide<HOPF_NT, 6>;
    case 8: return k_pdhg_wide<HOPF_NT, 8>;
    case 10: return k_pdhg_wide<HOPF_NT, 10>;
    case 12: return k_pdhg_wide<HOPF_NT, 12>;
    case 16: return k_pdhg_wide<HOPF_NT, 16>;
    default: return nullptr;
  }
#endif
}

pdhg_fn HOPF_CAT(stream_lookup_nt, HOPF_NT)(int bf16) {
  return bf16 ? k_pdhg_stream<HOPF_NT, true> : k_pdhg_stream<HOPF_NT, false>;
}

pdhg_fn HOPF_CAT(swide_lookup_nt, HOPF_NT)(int bf16) {
  return bf16 ? k_pdhg_swide<HOPF_NT, true> : k_pdhg_swide<HOPF_NT, false>;
}

cert_fn HOPF_CAT(cert_lookup_nt, HOPF_NT)() { return k_certify<HOPF_NT>; }

}  // namespace hopf
