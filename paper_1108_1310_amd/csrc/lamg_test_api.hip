// Inspection and per-kernel entry points (include/lamg_test.h).
#include <algorithm>
#include <cstring>
#include <vector>

#include "../../include/lamg_test.h"
#include "lamg_internal.hpp"
#include "lamg_sort.hpp"

using namespace lamg;


namespace {
template <class T>
void d2h(T* dst, const T* src, size_t n) {
  if (dst && src && n) LAMG_HIP(hipMemcpy(dst, src, n * sizeof(T), hipMemcpyDeviceToHost));
}
lamg_status guard(lamg_handle h, int l) {
  if (!h || l < 0 || l >= (int)h->H.lv.size()) return LAMG_E_INVALID_ARG;
  return LAMG_OK;
}
// A throwaway hierarchy holding one caller-provided level (device arrays are
// borrowed; only the tiles are allocated and freed here).
struct Scratch {
  Hierarchy H;
  ~Scratch() {
    (void)hipStreamSynchronize(H.s);
    for (void* p : H.owned) dev_free(H.o, p);
  }
};
Level borrowed_level(Scratch& S, int n, const int32_t* rp, const int32_t* ci, int ncol, const int32_t* cptr) {
  Level L;
  L.n = n;
  L.rp = (int*)rp;
  L.ci = (int*)ci;
  L.ncol = ncol;
  L.cptr.assign(cptr, cptr + ncol + 1);
  build_tiles(&S.H, L);
  return L;
}
// Device temporaries of one test call.
struct DevTmp {
  void* p = nullptr;
  explicit DevTmp(size_t bytes) { LAMG_HIP(hipMalloc(&p, std::max<size_t>(bytes, 16))); }
  ~DevTmp() { (void)hipFree(p); }
};
template <class K, class V>
lamg_status sort_entry(int64_t n, const K* k, const V* v, K* ko, V* vo, int endbit) {
  if (n < 0 || (n > 0 && (!k || !ko)) || endbit < 1 || endbit > (int)(8 * sizeof(K))) return LAMG_E_INVALID_ARG;
  if (n == 0) return LAMG_OK;
  try {
    DevTmp t(sortk::sort_scratch_bytes<K, V>(n));
    sortk::radix_sort<K, V>(nullptr, k, ko, v, vo, n, (unsigned)endbit, t.p);
    LAMG_HIP(hipGetLastError());
    LAMG_HIP(hipStreamSynchronize(nullptr));
  } catch (const DevError&) {
    return LAMG_E_DEVICE;
  }
  return LAMG_OK;
}
}  // namespace

extern "C" {

lamg_status lamg_t_sort_pairs64(int64_t n, const uint64_t* keys, const double* vals, uint64_t* keys_out,
                                double* vals_out, int32_t endbit) {
  if (n > 0 && (!vals || !vals_out)) return LAMG_E_INVALID_ARG;
  return sort_entry<uint64_t, double>(n, keys, vals, keys_out, vals_out, endbit);
}
lamg_status lamg_t_sort_pairs32(int64_t n, const uint32_t* keys, const int32_t* vals, uint32_t* keys_out,
                                int32_t* vals_out, int32_t endbit) {
  if (n > 0 && (!vals || !vals_out)) return LAMG_E_INVALID_ARG;
  return sort_entry<uint32_t, int32_t>(n, keys, vals, keys_out, vals_out, endbit);
}
lamg_status lamg_t_sort_f64(int64_t n, const double* keys, double* keys_out) {
  return sort_entry<double, sortk::NoVal>(n, keys, nullptr, keys_out, nullptr, 64);
}
lamg_status lamg_t_excl_scan(int64_t n, const int32_t* in, int32_t* out) {
  if (n < 0 || !out || (n > 0 && !in)) return LAMG_E_INVALID_ARG;
  try {
    DevTmp t(sortk::scan_scratch(n) * sizeof(int));
    sortk::exclusive_scan(nullptr, in, out, n, (int*)t.p);
    LAMG_HIP(hipGetLastError());
    LAMG_HIP(hipStreamSynchronize(nullptr));
  } catch (const DevError&) {
    return LAMG_E_DEVICE;
  }
  return LAMG_OK;
}

int lamg_t_num_levels(lamg_handle h) { return h ? (int)h->H.lv.size() : 0; }
int lamg_t_coarsest_relax(lamg_handle h) { return h && h->H.coarsest_relax ? 1 : 0; }

lamg_status lamg_t_level_dims(lamg_handle h, int l, int64_t* d) {
  if (guard(h, l) != LAMG_OK || !d) return LAMG_E_INVALID_ARG;
  const Level& L = h->H.lv[l];
  d[0] = L.n; d[1] = L.nnz; d[2] = L.type; d[3] = L.ncol; d[4] = L.nF; d[5] = L.K; d[6] = L.stage;
  d[7] = L.all.nlong;
  return LAMG_OK;
}

double lamg_t_level_gamma(lamg_handle h, int l) {
  if (guard(h, l) != LAMG_OK) return 0.0;
  return h->H.lv[l].gamma_next;
}

lamg_status lamg_t_level_export(lamg_handle h, int l, int32_t* rp, int32_t* ci, double* val, double* diag,
                                int32_t* cptr, int32_t* perm) {
  if (guard(h, l) != LAMG_OK) return LAMG_E_INVALID_ARG;
  try {
    const Level& L = h->H.lv[l];
    LAMG_HIP(hipStreamSynchronize(h->H.s));
    d2h(rp, L.rp, (size_t)L.n + 1);
    d2h(ci, L.ci, (size_t)L.nnz);
    d2h(val, L.val, (size_t)L.nnz);
    d2h(diag, L.diag, (size_t)L.n);
    if (cptr) std::copy(L.cptr.begin(), L.cptr.end(), cptr);
    d2h(perm, L.perm, (size_t)L.n);
  } catch (const DevError&) {
    return LAMG_E_DEVICE;
  }
  return LAMG_OK;
}

lamg_status lamg_t_transfer_export(lamg_handle h, int l, int32_t* out) {
  if (guard(h, l) != LAMG_OK || l == 0 || !out) return LAMG_E_INVALID_ARG;
  try {
    const Level& C = h->H.lv[l];
    const int nf = h->H.lv[l - 1].n;
    LAMG_HIP(hipStreamSynchronize(h->H.s));
    d2h(out, C.type == LT_AGG ? C.agg : C.cidx, (size_t)nf);
  } catch (const DevError&) {
    return LAMG_E_DEVICE;
  }
  return LAMG_OK;
}

lamg_status lamg_t_agg_export(lamg_handle h, int l, double* tv, double* aff, uint8_t* ok, uint8_t* weak, uint8_t* hub,
                              int32_t* state, double* scal) {
  if (guard(h, l) != LAMG_OK) return LAMG_E_INVALID_ARG;
  const Level& L = h->H.lv[l];
  if (!L.tv) return LAMG_E_INVALID_ARG;
  try {
    LAMG_HIP(hipStreamSynchronize(h->H.s));
    d2h(tv, L.tv, (size_t)L.n * L.K);
    d2h(aff, L.aff, (size_t)L.nnz);
    d2h(ok, L.ok, (size_t)L.nnz);
    d2h(weak, L.weak, (size_t)L.nnz);
    d2h(hub, L.hub, (size_t)L.n);
    d2h(state, L.state, (size_t)L.n);
    if (scal) { scal[0] = L.delta1; scal[1] = L.alpha1; scal[2] = L.alpha2; scal[3] = L.stage; scal[4] = L.rate; }
  } catch (const DevError&) {
    return LAMG_E_DEVICE;
  }
  return LAMG_OK;
}

lamg_status lamg_t_cycle(lamg_handle h, const double* b, double* x) {
  if (!h || !b || !x) return LAMG_E_INVALID_ARG;
  try {
    Hierarchy* H = &h->H;
    const int n = H->lv[0].n;
    Vecs<double>& v = H->lv[0].v64;
    LAMG_HIP(hipMemcpyAsync(v.b, b, n * sizeof(double), hipMemcpyDeviceToDevice, H->s));
    LAMG_HIP(hipMemcpyAsync(v.x, x, n * sizeof(double), hipMemcpyDeviceToDevice, H->s));
    cycle<double>(H);
    LAMG_HIP(hipMemcpyAsync(x, v.x, n * sizeof(double), hipMemcpyDeviceToDevice, H->s));
    LAMG_HIP(hipStreamSynchronize(H->s));
  } catch (const DevError&) {
    return LAMG_E_DEVICE;
  }
  return LAMG_OK;
}

lamg_status lamg_t_coarsest_solve(lamg_handle h, const double* b, double* x) {
  if (!h || !b || !x || h->H.coarsest_relax) return LAMG_E_INVALID_ARG;
  try {
    coarsest_solve(h->H.s, &h->H, b, x);
    LAMG_HIP(hipStreamSynchronize(h->H.s));
  } catch (const DevError&) {
    return LAMG_E_DEVICE;
  }
  return LAMG_OK;
}

lamg_status lamg_t_gs(int32_t n, const int32_t* rp, const int32_t* ci, const double* val, const double* diag,
                      int32_t ncol, const int32_t* cptr, const double* b, double* x, int32_t sweeps, void* stream) {
  if (n < 1 || !rp || !ci || !val || !diag || !x || ncol < 1 || !cptr || cptr[0] != 0 || cptr[ncol] != n)
    return LAMG_E_INVALID_ARG;
  try {
    Scratch S;
    S.H.s = (hipStream_t)stream;
    Level L = borrowed_level(S, n, rp, ci, ncol, cptr);
    for (int i = 0; i < sweeps; ++i) gs_sweep<double>(S.H.s, L, val, diag, b, x);
    LAMG_HIP(hipStreamSynchronize(S.H.s));
  } catch (const DevError&) {
    return LAMG_E_DEVICE;
  }
  return LAMG_OK;
}

lamg_status lamg_t_hub_info(lamg_handle h, int32_t l, int64_t* out) {
  if (!h || !out || l < 0 || l >= (int)h->H.lv.size()) return LAMG_E_INVALID_ARG;
  const Level& L = h->H.lv[l];
  out[0] = L.hub_k;
  out[1] = L.hub_k >= 0 ? L.hub_r0 : 0;
  out[2] = L.hub_k >= 0 ? L.hub_n : 0;
  out[3] = L.hub_k >= 0 ? L.hub_nnz : 0;
  return LAMG_OK;
}

lamg_status lamg_t_level_gs(lamg_handle h, int32_t l, int32_t precision, int32_t sweeps, const void* b, void* x) {
  if (!h || !x || l < 0 || l >= (int)h->H.lv.size() || sweeps < 0 || (precision != 0 && precision != 1))
    return LAMG_E_INVALID_ARG;
  try {
    Hierarchy* H = &h->H;
    const Level& L = H->lv[l];
    for (int i = 0; i < sweeps; ++i) {
      if (precision == 0) gs_sweep<double>(H->s, L, L.val, L.diag, (const double*)b, (double*)x);
      else gs_sweep<float>(H->s, L, L.val32, L.diag32, (const float*)b, (float*)x);
    }
    LAMG_HIP(hipStreamSynchronize(H->s));
  } catch (const DevError& e) {
    set_last_error("lamg_t_level_gs", e.e);
    return LAMG_E_DEVICE;
  }
  return LAMG_OK;
}

lamg_status lamg_t_level_gs_zero(lamg_handle h, int32_t l, int32_t precision, int32_t sweeps, const void* b,
                                 void* x) {
  if (!h || !x || l < 0 || l >= (int)h->H.lv.size() || sweeps < 1 || (precision != 0 && precision != 1))
    return LAMG_E_INVALID_ARG;
  try {
    Hierarchy* H = &h->H;
    const Level& L = H->lv[l];
    const size_t bytes = (size_t)L.n * (precision == 0 ? sizeof(double) : sizeof(float));
    LAMG_HIP(hipMemsetAsync(x, 0, bytes, H->s));
    for (int i = 0; i < sweeps; ++i) {
      if (precision == 0) gs_sweep<double>(H->s, L, L.val, L.diag, (const double*)b, (double*)x, i == 0);
      else gs_sweep<float>(H->s, L, L.val32, L.diag32, (const float*)b, (float*)x, i == 0);
    }
    LAMG_HIP(hipStreamSynchronize(H->s));
  } catch (const DevError& e) {
    set_last_error("lamg_t_level_gs_zero", e.e);
    return LAMG_E_DEVICE;
  }
  return LAMG_OK;
}

lamg_status lamg_t_gs32(int32_t n, const int32_t* rp, const int32_t* ci, const float* val, const float* diag,
                        int32_t ncol, const int32_t* cptr, const float* b, float* x, int32_t sweeps, void* stream) {
  if (n < 1 || !rp || !ci || !val || !diag || !x || ncol < 1 || !cptr || cptr[0] != 0 || cptr[ncol] != n)
    return LAMG_E_INVALID_ARG;
  try {
    Scratch S;
    S.H.s = (hipStream_t)stream;
    Level L = borrowed_level(S, n, rp, ci, ncol, cptr);
    for (int i = 0; i < sweeps; ++i) gs_sweep<float>(S.H.s, L, val, diag, b, x);
    LAMG_HIP(hipStreamSynchronize(S.H.s));
  } catch (const DevError&) {
    return LAMG_E_DEVICE;
  }
  return LAMG_OK;
}

lamg_status lamg_t_residual(int32_t n, const int32_t* rp, const int32_t* ci, const double* val, const double* diag,
                            const double* b, const double* x, double* r, void* stream) {
  if (n < 1 || !rp || !ci || !val || !diag || !b || !x || !r) return LAMG_E_INVALID_ARG;
  try {
    Scratch S;
    S.H.s = (hipStream_t)stream;
    int32_t cp[2] = {0, n};
    Level L = borrowed_level(S, n, rp, ci, 1, cp);
    residual<double>(S.H.s, L, val, diag, b, x, r);
    LAMG_HIP(hipStreamSynchronize(S.H.s));
  } catch (const DevError&) {
    return LAMG_E_DEVICE;
  }
  return LAMG_OK;
}

lamg_status lamg_t_colour(int32_t n, const int32_t* rp, const int32_t* ci, uint64_t seed, int32_t level,
                          int32_t* colour, void* stream) {
  if (n < 1 || !rp || !ci || !colour) return LAMG_E_INVALID_ARG;
  try {
    colour_greedy((hipStream_t)stream, n, rp, ci, seed, level, colour);
    LAMG_HIP(hipStreamSynchronize((hipStream_t)stream));
  } catch (const DevError&) {
    return LAMG_E_DEVICE;
  }
  return LAMG_OK;
}

}  // extern "C"
