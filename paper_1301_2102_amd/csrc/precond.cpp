// IC(0) preconditioner: the caller-owned device buffer, its symbolic set-up
// and the triangular-solve entry point (see include/bmr.h).
//
// The set-up reads the pattern of M once on the host (integer work only:
// the strictly lower pattern, the position of every entry in M's arrays, the
// level of every row and the transposed pattern) and writes it into the
// buffer; the numeric factorisation and every solve run on the device
// (kernels_ic0.hip).
#include <string.h>

#include <algorithm>
#include <vector>

#include "bmr_internal.hpp"

namespace bmr {
namespace {

constexpr uint64_t IC0_MAGIC = 0x3043494d52423032ull;  // "BMRIC0" tag and layout version

// Header at the start of the buffer; the arrays follow at the recorded
// offsets (bytes from the start, 256-byte aligned).
struct Ic0Header {
  uint64_t magic;
  int64_t n, nnz_l, n_levels;
  uint64_t off_level_ptr, off_level_rows, off_lrp, off_lci, off_lmap, off_dmap, off_lval;
  uint64_t off_urp, off_uci, off_upos, off_uval, off_diag, off_lval_s, off_uval_s, off_fail, total;
};

size_t a256(size_t x) { return (x + 255) & ~size_t(255); }

// Offsets for n rows and at most nnz_l strictly lower entries (n_levels <= n).
Ic0Header plan(int64_t n, int64_t nnz_l) {
  Ic0Header h{};
  size_t o = a256(sizeof(Ic0Header));
  auto take = [&](uint64_t& field, size_t bytes) {
    field = o;
    o = a256(o + bytes);
  };
  take(h.off_level_ptr, sizeof(int32_t) * (size_t)(n + 1));
  take(h.off_level_rows, sizeof(int32_t) * (size_t)n);
  take(h.off_lrp, sizeof(int32_t) * (size_t)(n + 1));
  take(h.off_lci, sizeof(int32_t) * (size_t)nnz_l);
  take(h.off_lmap, sizeof(int32_t) * (size_t)nnz_l);
  take(h.off_dmap, sizeof(int32_t) * (size_t)n);
  take(h.off_lval, sizeof(double) * (size_t)nnz_l);
  take(h.off_urp, sizeof(int32_t) * (size_t)(n + 1));
  take(h.off_uci, sizeof(int32_t) * (size_t)nnz_l);
  take(h.off_upos, sizeof(int32_t) * (size_t)nnz_l);
  take(h.off_uval, sizeof(double) * (size_t)nnz_l);
  take(h.off_diag, sizeof(double) * (size_t)n);
  take(h.off_lval_s, sizeof(double) * (size_t)nnz_l);
  take(h.off_uval_s, sizeof(double) * (size_t)nnz_l);
  take(h.off_fail, sizeof(int));
  h.total = o;
  h.magic = IC0_MAGIC;
  h.n = n;
  h.nnz_l = nnz_l;
  return h;
}

bool csr_ok(const bmr_csr_t* A) {
  return A && A->n >= 1 && A->n < (int64_t(1) << 31) && A->nnz >= 0 && A->nnz < (int64_t(1) << 31) &&
         A->row_ptr && (A->nnz == 0 || (A->col_idx && A->val));
}

#define HTRY(expr)                              \
  do {                                          \
    if ((expr) != hipSuccess) return BMR_HIP_ERROR; \
  } while (0)

}  // namespace

int ic0_view(const void* buf, Ic0View* v) {
  Ic0Header h;
  HTRY(hipMemcpy(&h, buf, sizeof(h), hipMemcpyDeviceToHost));
  if (h.magic != IC0_MAGIC || h.n < 1 || h.n_levels < 1 || h.n_levels > h.n) return BMR_INVALID_ARG;
  const char* b = (const char*)buf;
  v->n = h.n;
  v->nnz_l = h.nnz_l;
  v->n_levels = (int)h.n_levels;
  v->level_ptr.resize((size_t)h.n_levels + 1);
  HTRY(hipMemcpy(v->level_ptr.data(), b + h.off_level_ptr, sizeof(int32_t) * v->level_ptr.size(),
                 hipMemcpyDeviceToHost));
  v->level_rows = (const int32_t*)(b + h.off_level_rows);
  v->lrp = (const int32_t*)(b + h.off_lrp);
  v->lci = (const int32_t*)(b + h.off_lci);
  v->lmap = (const int32_t*)(b + h.off_lmap);
  v->dmap = (const int32_t*)(b + h.off_dmap);
  v->lval = (double*)(b + h.off_lval);
  v->urp = (const int32_t*)(b + h.off_urp);
  v->uci = (const int32_t*)(b + h.off_uci);
  v->upos = (const int32_t*)(b + h.off_upos);
  v->uval = (double*)(b + h.off_uval);
  v->diag = (double*)(b + h.off_diag);
  v->lval_s = (double*)(b + h.off_lval_s);
  v->uval_s = (double*)(b + h.off_uval_s);
  v->fail = (int*)(b + h.off_fail);
  return 0;
}

}  // namespace bmr

using namespace bmr;

extern "C" {

int bmr_ic0_bytes(int64_t n, int64_t nnz, size_t* bytes) {
  if (!bytes || n < 1 || n >= (int64_t(1) << 31) || nnz < 0 || nnz >= (int64_t(1) << 31)) return BMR_INVALID_ARG;
  *bytes = plan(n, nnz).total;
  return BMR_CONVERGED;
}

int bmr_ic0_factor(const bmr_csr_t* M, void* buf, size_t bytes, hipStream_t stream) {
  if (!csr_ok(M) || !buf || ((uintptr_t)buf & 255u) != 0) return BMR_INVALID_ARG;
  const int64_t n = M->n, nnz = M->nnz;
  if (bytes < plan(n, nnz).total) return BMR_WORKSPACE_TOO_SMALL;
  // the pattern of M on the host
  std::vector<int32_t> rp((size_t)n + 1), ci((size_t)nnz);
  HTRY(hipMemcpyAsync(rp.data(), M->row_ptr, sizeof(int32_t) * rp.size(), hipMemcpyDeviceToHost, stream));
  if (nnz > 0)
    HTRY(hipMemcpyAsync(ci.data(), M->col_idx, sizeof(int32_t) * ci.size(), hipMemcpyDeviceToHost, stream));
  HTRY(hipStreamSynchronize(stream));
  if (rp[0] != 0 || rp[n] != nnz) return BMR_INVALID_ARG;
  // strictly lower pattern (columns ascending), positions in M, diagonal positions
  std::vector<int32_t> lrp((size_t)n + 1, 0), lci, lmap, dmap((size_t)n, -1), level((size_t)n, 0);
  lci.reserve((size_t)(nnz / 2 + 1));
  lmap.reserve((size_t)(nnz / 2 + 1));
  int32_t n_levels = 1;
  for (int64_t i = 0; i < n; ++i) {
    if (rp[i + 1] < rp[i]) return BMR_INVALID_ARG;
    int32_t lev = 0, prev = -1;
    for (int32_t q = rp[i]; q < rp[i + 1]; ++q) {
      const int32_t j = ci[q];
      if (j <= prev || j < 0 || j >= n) return BMR_INVALID_ARG;  // columns sorted, unique, in range
      prev = j;
      if (j < i) {
        lci.push_back(j);
        lmap.push_back(q);
        lev = std::max(lev, level[j] + 1);
      } else if (j == i) {
        dmap[i] = q;
      }
    }
    if (dmap[i] < 0) return BMR_INVALID_ARG;  // IC(0) needs every diagonal entry
    level[i] = lev;
    n_levels = std::max(n_levels, lev + 1);
    lrp[i + 1] = (int32_t)lci.size();
  }
  const int64_t nnz_l = (int64_t)lci.size();
  // rows by level (ascending row index within a level)
  std::vector<int32_t> level_ptr((size_t)n_levels + 1, 0), level_rows((size_t)n);
  for (int64_t i = 0; i < n; ++i) ++level_ptr[level[i] + 1];
  for (int32_t l = 0; l < n_levels; ++l) level_ptr[l + 1] += level_ptr[l];
  {
    std::vector<int32_t> fill(level_ptr.begin(), level_ptr.end() - 1);
    for (int64_t i = 0; i < n; ++i) level_rows[fill[level[i]]++] = (int32_t)i;
  }
  // transpose of the strictly lower part: row j of it lists the rows i > j
  // with an entry (i, j), ascending, with that entry's position
  std::vector<int32_t> urp((size_t)n + 1, 0), uci((size_t)nnz_l), upos((size_t)nnz_l);
  for (int64_t e = 0; e < nnz_l; ++e) ++urp[lci[e] + 1];
  for (int64_t j = 0; j < n; ++j) urp[j + 1] += urp[j];
  {
    std::vector<int32_t> fill(urp.begin(), urp.end() - 1);
    for (int64_t i = 0; i < n; ++i)
      for (int32_t e = lrp[i]; e < lrp[i + 1]; ++e) {
        const int32_t at = fill[lci[e]]++;
        uci[at] = (int32_t)i;
        upos[at] = e;
      }
  }
  Ic0Header h = plan(n, nnz);
  h.nnz_l = nnz_l;
  h.n_levels = n_levels;
  char* b = (char*)buf;
  const int zero = 0;
  auto put = [&](uint64_t off, const void* src, size_t sz) -> int {
    if (sz) HTRY(hipMemcpyAsync(b + off, src, sz, hipMemcpyHostToDevice, stream));
    return 0;
  };
  if (put(0, &h, sizeof(h)) || put(h.off_level_ptr, level_ptr.data(), 4 * level_ptr.size()) ||
      put(h.off_level_rows, level_rows.data(), 4 * level_rows.size()) || put(h.off_lrp, lrp.data(), 4 * lrp.size()) ||
      put(h.off_lci, lci.data(), 4 * lci.size()) || put(h.off_lmap, lmap.data(), 4 * lmap.size()) ||
      put(h.off_dmap, dmap.data(), 4 * dmap.size()) || put(h.off_urp, urp.data(), 4 * urp.size()) ||
      put(h.off_uci, uci.data(), 4 * uci.size()) || put(h.off_upos, upos.data(), 4 * upos.size()) ||
      put(h.off_fail, &zero, sizeof(int)))
    return BMR_HIP_ERROR;
  HTRY(hipStreamSynchronize(stream));  // the host vectors go out of scope below
  Ic0View v;
  const int e = ic0_view(buf, &v);
  if (e) return e;
  HTRY(launch_ic0_factor(v, M->val, v.fail, stream));
  int fail = 0;
  HTRY(hipMemcpyAsync(&fail, v.fail, sizeof(int), hipMemcpyDeviceToHost, stream));
  HTRY(hipStreamSynchronize(stream));
  return fail ? BMR_IC0_BREAKDOWN : BMR_CONVERGED;
}

int bmr_ic0_apply(const void* ic0, const double* V, double* W, int p, int trans, hipStream_t stream) {
  if (!ic0 || !V || !W || p < 1 || p > BMR_MAX_P) return BMR_INVALID_ARG;
  Ic0View v;
  const int e = ic0_view(ic0, &v);
  if (e) return e;
  HTRY(launch_ic0_solve(v, p, trans != 0, V, W, nullptr, stream));
  return BMR_CONVERGED;
}

}  // extern "C"
