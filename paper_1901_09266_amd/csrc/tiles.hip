// Host construction of the dense MFMA tiles of the assignment blocks.
//
// Every lag block rho_c[l][t] (L links x P ODs, eq. "assign") shares one
// incidence pattern.  For the forward product a tile row is 16 consecutive
// links and its columns are the contiguous OD range that covers the ODs of
// those links (padded to whole 32-wide k-steps); for the adjoint a tile row is
// 16 consecutive ODs and its columns the covering link range.  Entries of the
// range that are not in the pattern hold zero.  With ODs sorted along their
// corridor the ranges are short, so most of the empty area of a block is
// never stored or multiplied.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "dode_internal.h"

namespace {

int32_t round_up(int32_t x, int32_t m) { return (x + m - 1) / m * m; }

struct Hull {
  int32_t lo = 0, ks = 0;
};

// Covering ranges of `n_rows` rows grouped by 16, given per-row sorted column
// lists; the tiles of each run of `group` consecutive tiles share the range
// that covers all of them (one wave multiplies them with the same operand).
std::vector<Hull> hulls(int32_t n_rows, int32_t n_cols, const std::vector<int32_t>& ptr,
                        const std::vector<int32_t>& idx, int32_t group) {
  const int32_t nt = (n_rows + 15) / 16;
  std::vector<Hull> out(nt);
  for (int32_t i = 0; i < nt; ++i) {
    const int32_t g0 = i / group * group;
    int32_t lo = n_cols, hi = 0;
    for (int32_t r = 16 * g0; r < std::min(n_rows, 16 * (g0 + group)); ++r)
      if (ptr[r + 1] > ptr[r]) {
        lo = std::min(lo, idx[ptr[r]]);
        hi = std::max(hi, idx[ptr[r + 1] - 1] + 1);
      }
    if (hi <= lo) continue;
    lo = lo / 8 * 8;   // starts on a multiple of 8 columns (32-byte FP32 operand loads)
    const int32_t len = round_up(hi - lo, 32);
    if (lo + len > n_cols && len <= n_cols) {
      // move the range left to stay inside [0, n_cols) when it still covers [lo, hi)
      const int32_t lo2 = (n_cols - len) / 8 * 8;
      if (lo2 + len >= hi) lo = lo2;
    }
    out[i].lo = lo;
    out[i].ks = len / 32;
  }
  return out;
}

// Position of a (row, col) entry inside the packed k-steps of its row tile.
// Within a 32-wide k-step, lane group g (lanes 16g..16g+15) holds columns
// 4g..4g+3 (elements 0-3) and 16+4g..16+4g+3 (elements 4-7): the FP32 operand
// the kernels pair with it is then read as two 64-byte runs per row.
int64_t packed_pos(int32_t row, int32_t col, const std::vector<Hull>& hs,
                   const std::vector<int32_t>& koff) {
  const int32_t i = row / 16, m = row % 16;
  const int32_t k = col - hs[i].lo;
  const int32_t ks = k / 32, kk = k % 32;
  const int32_t half = kk / 16, g = (kk % 16) / 4;
  const int32_t lane = m + 16 * g, e = 4 * half + kk % 4;
  return ((int64_t)(koff[i] + ks) * 64 + lane) * 8 + e;
}

}  // namespace

dode_status tiles_prepare(dode_dar* d, std::string& err) {
  const dode_dims& dm = d->dims;
  const int64_t nnz = d->nnz;
  const std::vector<Hull> fh = hulls(dm.L, dm.P, d->h_row_ptr, d->h_col, kFwdTileGroup);
  const std::vector<Hull> gh = hulls(dm.P, dm.L, d->h_col_ptr, d->h_row, 1);
  const int32_t nLT = (int32_t)fh.size(), nPT = (int32_t)gh.size();
  std::vector<int32_t> meta;
  std::vector<int32_t> fko(nLT + 1, 0), gko(nPT + 1, 0);
  for (int32_t i = 0; i < nLT; ++i) fko[i + 1] = fko[i] + fh[i].ks;
  for (int32_t j = 0; j < nPT; ++j) gko[j + 1] = gko[j] + gh[j].ks;
  for (auto& h : fh) meta.push_back(h.lo);
  for (auto& h : fh) meta.push_back(h.ks);
  for (int32_t i = 0; i < nLT; ++i) meta.push_back(fko[i]);
  for (auto& h : gh) meta.push_back(h.lo);
  for (auto& h : gh) meta.push_back(h.ks);
  for (int32_t j = 0; j < nPT; ++j) meta.push_back(gko[j]);
  const int32_t kf = fko[nLT], kg = gko[nPT];

  // packed position of every pattern entry, forward (CSR slot j) and adjoint (CSC slot jj)
  auto inside = [](int32_t col, const Hull& h) { return col >= h.lo && col < h.lo + 32 * h.ks; };
  d->h_posf.resize(nnz);
  d->h_posg.resize(nnz);
  for (int32_t a = 0; a < dm.L; ++a)
    for (int32_t j = d->h_row_ptr[a]; j < d->h_row_ptr[a + 1]; ++j) {
      if (!inside(d->h_col[j], fh[a / 16])) {
        err = "internal: forward tile range misses a pattern entry";
        return DODE_ERR_SHAPE;
      }
      d->h_posf[j] = (int32_t)packed_pos(a, d->h_col[j], fh, fko);
    }
  for (int32_t p = 0; p < dm.P; ++p)
    for (int32_t jj = d->h_col_ptr[p]; jj < d->h_col_ptr[p + 1]; ++jj) {
      if (!inside(d->h_row[jj], gh[p / 16])) {
        err = "internal: adjoint tile range misses a pattern entry";
        return DODE_ERR_SHAPE;
      }
      d->h_posg[jj] = (int32_t)packed_pos(p, d->h_row[jj], gh, gko);
    }
  auto hip_ok = [&](hipError_t e) {
    if (e != hipSuccess) err = hipGetErrorString(e);
    return e == hipSuccess;
  };
  auto up = [&](int32_t** dst, const std::vector<int32_t>& v) -> bool {
    if (!hip_ok(hipMalloc(dst, std::max<size_t>(16, v.size() * 4)))) return false;
    return hip_ok(hipMemcpy(*dst, v.data(), v.size() * 4, hipMemcpyHostToDevice));
  };
  d->h_tile_meta = meta;
  if (!up(&d->d_tile_meta, meta) || !up(&d->d_posf, d->h_posf) || !up(&d->d_posg, d->h_posg))
    return DODE_ERR_OOM;
  const size_t esz = d->storage == DODE_FP8_E4M3 ? 1 : 2;
  const int64_t blocks = (int64_t)dm.K * dm.T;
  const size_t fbytes = (size_t)d->C * blocks * kf * 512 * esz;
  const size_t gbytes = (size_t)d->C * blocks * kg * 512 * esz;
  if (!hip_ok(hipMalloc(&d->d_Fv, std::max<size_t>(16, fbytes)))) return DODE_ERR_OOM;
  if (!hip_ok(hipMalloc(&d->d_Gv, std::max<size_t>(16, gbytes)))) return DODE_ERR_OOM;
  d->device_bytes += fbytes + gbytes + meta.size() * 4 + 8 * nnz;
  if (d->has_corr) {
    // bf16 correction tiles, 2 bytes per entry whatever the storage type
    const size_t cf = fbytes / esz * 2, cg = gbytes / esz * 2;
    if (!hip_ok(hipMalloc(&d->d_Fc, std::max<size_t>(16, cf)))) return DODE_ERR_OOM;
    if (!hip_ok(hipMalloc(&d->d_Gc, std::max<size_t>(16, cg)))) return DODE_ERR_OOM;
    d->device_bytes += cf + cg;
  }
  DevTiles& T = d->tiles;
  T.nLT = nLT;
  T.nPT = nPT;
  T.kf_total = kf;
  T.kg_total = kg;
  const int32_t* m = d->d_tile_meta;
  T.f_plo = m;
  T.f_ks = m + nLT;
  T.f_koff = m + 2 * nLT;
  T.g_alo = m + 3 * nLT;
  T.g_ks = m + 3 * nLT + nPT;
  T.g_koff = m + 3 * nLT + 2 * nPT;
  T.Fv = d->d_Fv;
  T.Gv = d->d_Gv;
  T.scale = d->d_scale;
  T.n_ptile = (dm.P + 63) / 64;
  T.Fc = d->d_Fc;
  T.Gc = d->d_Gc;
  d->has_tiles = true;
  return DODE_OK;
}

namespace {

// Scatter one cluster's codes (CSR order, esz bytes each) into packed forward
// tiles F and adjoint tiles G.
template <typename E>
dode_status fill_tiles(dode_dar* d, int32_t c, const E* codes_csr, void* F, void* G,
                       std::string& err) {
  const dode_dims& dm = d->dims;
  const int64_t nnz = d->nnz;
  const int64_t blocks = (int64_t)dm.K * dm.T;
  const size_t fblk = (size_t)d->tiles.kf_total * 512, gblk = (size_t)d->tiles.kg_total * 512;
  std::vector<E> fbuf(blocks * fblk, E(0)), gbuf(blocks * gblk, E(0));
  host_parallel_for(blocks, [&](int64_t b0, int64_t b1) {
    for (int64_t lt = b0; lt < b1; ++lt) {
      const int32_t l = (int32_t)(lt / dm.T), t = (int32_t)(lt % dm.T);
      if (t + l >= dm.H) continue;   // block past the last interval: never read
      const E* w = codes_csr + lt * nnz;
      E* fb = fbuf.data() + lt * fblk;
      E* gb = gbuf.data() + lt * gblk;
      for (int64_t j = 0; j < nnz; ++j) fb[d->h_posf[j]] = w[j];
      for (int64_t jj = 0; jj < nnz; ++jj) gb[d->h_posg[jj]] = w[d->h_csc2csr[jj]];
    }
  });
  hipError_t e = hipMemcpy(static_cast<E*>(F) + (size_t)c * blocks * fblk, fbuf.data(),
                           fbuf.size() * sizeof(E), hipMemcpyHostToDevice);
  if (e == hipSuccess)
    e = hipMemcpy(static_cast<E*>(G) + (size_t)c * blocks * gblk, gbuf.data(),
                  gbuf.size() * sizeof(E), hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    err = hipGetErrorString(e);
    return DODE_ERR_HIP;
  }
  return DODE_OK;
}

}  // namespace

dode_status tiles_fill_cluster(dode_dar* d, int32_t c, const void* codes_csr, std::string& err) {
  if (d->storage == DODE_FP8_E4M3)
    return fill_tiles(d, c, static_cast<const uint8_t*>(codes_csr), d->d_Fv, d->d_Gv, err);
  return fill_tiles(d, c, static_cast<const uint16_t*>(codes_csr), d->d_Fv, d->d_Gv, err);
}

dode_status tiles_fill_correction(dode_dar* d, int32_t c, const uint16_t* corr_csr,
                                  std::string& err) {
  return fill_tiles(d, c, corr_csr, d->d_Fc, d->d_Gc, err);
}
