// Checks of the host-only planning code (descriptor validation, stored-mode
// set, tiled slot layout, binning table, workspace layout, pair launch
// groups, twiddle table), built with g++ under AddressSanitizer and
// UndefinedBehaviorSanitizer by tests/test_host_sanitized.py. Exits non-zero
// on the first failed check.
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <set>
#include <string>
#include <utility>
#include <vector>

#include "nfs_host.hpp"

namespace {

int g_checks = 0;

void check(bool ok, const char* what, const std::string& ctx = "") {
  ++g_checks;
  if (!ok) {
    std::fprintf(stderr, "FAILED: %s %s\n", what, ctx.c_str());
    std::exit(1);
  }
}

nfs_desc make_desc(int n, const std::vector<int32_t>& lags, int n_bins, int64_t capacity) {
  nfs_desc d{};
  d.n = n;
  d.in_dtype = NFS_IN_U16;
  d.spec_dtype = NFS_SPEC_F32;
  d.accum = NFS_ACC_PLAIN;
  d.n_lags = int32_t(lags.size());
  d.lags = lags.empty() ? nullptr : lags.data();
  d.n_bins = n_bins;
  d.capacity = capacity;
  return d;
}

void check_integer_roots() {
  for (uint64_t v = 0; v < 200000; ++v) {
    const uint64_t s = nfs::isqrt_u64(v);
    check(s * s <= v && (s + 1) * (s + 1) > v, "isqrt_u64", std::to_string(v));
  }
  for (uint64_t s = (1u << 26) - 50; s < (1u << 26) + 50; ++s)
    for (int d = -1; d <= 1; ++d) {
      const uint64_t v = s * s + uint64_t(int64_t(d));
      const uint64_t r = nfs::isqrt_u64(v);
      check(r * r <= v && (r + 1) * (r + 1) > v, "isqrt_u64 near 2^52", std::to_string(v));
    }
  for (int64_t v = -3; v < 100000; ++v) {
    const int64_t s = nfs::ceil_sqrt_i64(v);
    check(s >= 0 && (v <= 0 ? s == 0 : (s * s >= v && (s - 1) * (s - 1) < v)), "ceil_sqrt",
          std::to_string(v));
  }
}

void check_bins() {
  for (int n : {16, 64, 256}) {
    for (int nb : {1, 3, n / 4, n / 2}) {
      const int h = n / 2;
      for (int ky = -h; ky < h; ++ky)
        for (int kx = 0; kx <= h; ++kx) {
          const int b = nfs::bin_of(n, nb, ky, kx);
          // b is the largest integer with (b h)^2 <= |k|^2 nb^2, or -1 when >= nb.
          const uint64_t k2 = uint64_t(ky * ky + kx * kx) * uint64_t(nb) * uint64_t(nb);
          uint64_t want = 0;
          while (uint64_t(want + 1) * h * uint64_t(want + 1) * h <= k2) ++want;
          check(b == (want < uint64_t(nb) ? int(want) : -1), "bin_of",
                std::to_string(n) + " " + std::to_string(ky) + "," + std::to_string(kx));
        }
    }
  }
}

void check_validation() {
  std::string err;
  std::vector<int32_t> lags = {1, 2, 4};
  check(nfs::validate_desc(nullptr, &err) == NFS_E_ARG, "null desc");
  nfs_desc d = make_desc(100, lags, 8, 16);
  check(nfs::validate_desc(&d, &err) == NFS_E_SIZE, "non power of two");
  d = make_desc(8, lags, 4, 16);
  check(nfs::validate_desc(&d, &err) == NFS_E_SIZE, "n too small");
  d = make_desc(8192, lags, 4, 16);
  check(nfs::validate_desc(&d, &err) == NFS_E_SIZE, "n too large");
  d = make_desc(64, lags, 33, 16);
  check(nfs::validate_desc(&d, &err) == NFS_E_BINS, "too many bins");
  d = make_desc(64, lags, 0, 16);
  check(nfs::validate_desc(&d, &err) == NFS_E_BINS, "zero bins");
  std::vector<int32_t> none;
  d = make_desc(64, none, 8, 16);
  check(nfs::validate_desc(&d, &err) == NFS_E_LAGS, "no lags");
  std::vector<int32_t> unsorted = {3, 1};
  d = make_desc(64, unsorted, 8, 16);
  check(nfs::validate_desc(&d, &err) == NFS_E_LAGS, "unsorted lags");
  std::vector<int32_t> dup = {1, 1};
  d = make_desc(64, dup, 8, 16);
  check(nfs::validate_desc(&d, &err) == NFS_E_LAGS, "duplicate lags");
  std::vector<int32_t> neg = {-1, 2};
  d = make_desc(64, neg, 8, 16);
  check(nfs::validate_desc(&d, &err) == NFS_E_LAGS, "negative lag");
  d = make_desc(64, lags, 8, 4);
  check(nfs::validate_desc(&d, &err) == NFS_E_CAPACITY, "capacity not above the largest lag");
  d = make_desc(64, lags, 8, -1);
  check(nfs::validate_desc(&d, &err) == NFS_E_CAPACITY, "negative capacity");
  d = make_desc(64, lags, 8, 16);
  d.spec_dtype = 7;
  check(nfs::validate_desc(&d, &err) == NFS_E_UNSUPPORTED, "bad spec");
  d = make_desc(64, lags, 8, 16);
  d.full_spectra = 2;
  check(nfs::validate_desc(&d, &err) == NFS_E_ARG, "bad full_spectra");
  d = make_desc(64, lags, 8, 16);
  check(nfs::validate_desc(&d, &err) == NFS_OK, "valid desc");
}

// Every invariant of one layout.
void check_layout(const nfs_desc& d, size_t bytes) {
  const std::string ctx = "n=" + std::to_string(d.n) + " L=" + std::to_string(d.n_lags) +
                          " cap=" + std::to_string(d.capacity) +
                          " full=" + std::to_string(d.full_spectra) +
                          " spec=" + std::to_string(d.spec_dtype) +
                          " bwd=" + std::to_string(d.backward);
  nfs::Layout L;
  std::string err;
  const nfs_status st = nfs::make_layout(&d, bytes, &L, &err);
  check(st == NFS_OK, "make_layout", ctx + " " + err);
  const int n = L.n, h = L.h;
  // Stored-mode set: the disc |k| < n/2 with k_x < n/2, or the half plane.
  int64_t disc = 0, stored = 0;
  for (int r = 0; r < n; ++r) {
    const int ky = r < h ? r : r - n;
    int w = 0;
    while (w < h && int64_t(ky) * ky + int64_t(w) * w < int64_t(h) * h) ++w;
    disc += w;
    check(L.row_width[size_t(r)] == (L.full ? h : w), "row width", ctx);
    stored += L.row_width[size_t(r)];
  }
  check(L.binned == disc, "binned modes", ctx);
  check(L.modes == stored + (L.full ? n : 0), "stored modes", ctx);
  // Slots: distinct, inside [0, slots), every stored mode has one.
  std::vector<char> used(size_t(L.slots), 0);
  for (int r = 0; r < n; ++r)
    for (int kx = 0; kx < L.row_width[size_t(r)]; ++kx) {
      const int s = nfs::ring_slot_host(L, r, kx);
      check(s >= 0 && s < L.slots && !used[size_t(s)], "slot bijection", ctx);
      used[size_t(s)] = 1;
    }
  if (L.full) {
    check(L.nyq_slot >= 0 && L.nyq_slot + n == L.slots, "Nyquist slots", ctx);
    for (int r = 0; r < n; ++r) {
      check(!used[size_t(L.nyq_slot + r)], "Nyquist slot free", ctx);
      used[size_t(L.nyq_slot + r)] = 1;
    }
  }
  check(L.mode_stride >= L.slots && L.mode_stride % 64 == 0, "mode stride", ctx);
  // Binning table: each disc mode once, weight bit = (k_x > 0), segments.
  check(int64_t(L.bin_slots.size()) == L.binned, "bin table size", ctx);
  std::set<int32_t> seen;
  for (int32_t e : L.bin_slots) {
    check(e >= 0 && (e >> 1) < L.slots && seen.insert(e >> 1).second, "bin table entry", ctx);
  }
  check(int(L.bin_seg0.size()) == L.n_bins + 1 && L.bin_seg0.front() == 0, "ring segments",
        ctx);
  for (size_t i = 0; i + 1 < L.seg_first.size(); ++i)
    check(L.seg_first[i + 1] > L.seg_first[i] &&
              L.seg_first[i + 1] - L.seg_first[i] <= nfs::kSegModes,
          "segment size", ctx);
  for (int b = 0; b < L.n_bins; ++b)
    check(L.bin_seg0[size_t(b) + 1] > L.bin_seg0[size_t(b)], "every ring has a segment", ctx);
  // Full-plane count of the disc from the weights.
  int64_t weighted = 0;
  for (int32_t e : L.bin_slots) weighted += (e & 1) ? 2 : 1;
  int64_t lattice = 0;
  for (int ky = -h; ky < h; ++ky)
    for (int kx = -h; kx < h; ++kx)
      if (int64_t(ky) * ky + int64_t(kx) * kx < int64_t(h) * h) ++lattice;
  check(weighted == lattice, "full-plane disc count", ctx);
  // Pair launch groups: contiguous cover of the lags, within the limits.
  int next = 0;
  for (const nfs::LagGroup& g : L.groups) {
    check(g.first == next && g.count >= 1, "group cover", ctx);
    check(g.max_lag == L.lags[size_t(g.first + g.count - 1)], "group max lag", ctx);
    if (g.modes == 0) {
      check(g.count <= nfs::kGlobalLags && L.lags[size_t(g.first)] > nfs::kMaxLag,
            "global group", ctx);
    } else {
      check(g.max_lag <= nfs::kMaxLag && (g.modes == 16 || g.modes == 8), "LDS group", ctx);
      check(g.lds <= size_t(nfs::kLdsBytes) && g.hist >= g.max_lag + 2 * nfs::kPairChunk,
            "LDS history", ctx);
      check(g.per_wave >= 1 && g.per_wave <= nfs::kMaxLagsPerWave &&
                g.waves * g.per_wave >= g.count && g.waves <= nfs::kMaxPairWaves,
            "wave split", ctx);
    }
    next = g.first + g.count;
  }
  check(next == L.n_lags, "groups cover every lag", ctx);
  // Workspace: aligned regions in order, the ring and its scales last.
  const std::vector<std::pair<const char*, size_t>> offs = {
      {"inter", L.off_inter}, {"rowsum", L.off_rowsum}, {"rowabs", L.off_rowabs},
      {"nyq", L.off_nyq},     {"acc", L.off_acc},       {"comp", L.off_comp},
      {"segs", L.off_segs},
      {"bin_slots", L.off_bin_slots}, {"part", L.off_part}, {"part_cnt", L.off_part_cnt},
      {"status", L.off_status}, {"tw", L.off_tw}, {"width", L.off_width},
      {"tiles", L.off_tiles}, {"lags", L.off_lags}, {"ref", L.off_ref},
      {"stage", L.off_stage}, {"refspec", L.off_refspec}, {"ring", L.off_ring},
      {"fscale", L.off_fscale}};
  size_t prev = 0;
  for (const auto& o : offs) {
    check(o.second % nfs::kAlign == 0, "aligned region", ctx + " " + o.first);
    check(o.second >= prev, "regions in order", ctx + " " + o.first);
    prev = o.second;
  }
  check(L.off_acc >= L.off_inter + size_t(L.batch) * n * h * 8, "intermediate size", ctx);
  check(L.off_comp >= L.off_acc + size_t(L.n_lags) * L.mode_stride * 4, "sums size", ctx);
  check(L.off_segs >= L.off_comp + (L.accum == NFS_ACC_KAHAN ? size_t(L.n_lags) * L.mode_stride * 4
                                                              : 0),
        "compensation size", ctx);
  check(L.off_fscale >= L.off_ring + size_t(L.capacity) * L.mode_stride * L.mode_bytes,
        "ring size", ctx);
  check(L.total >= L.off_fscale + size_t(L.capacity) * nfs::kScaleBytes, "total size", ctx);
  if (bytes) check(L.total <= bytes, "fits the workspace", ctx);
  check(L.capacity > L.max_lag, "capacity above the largest lag", ctx);
  // A given capacity bounds the transform batch; a derived one does not
  // (pushes are cut to capacity - largest lag frames at run time).
  check(L.batch >= 1 && (d.capacity == 0 || L.batch <= L.capacity - L.max_lag), "batch", ctx);
  if (L.backward) {
    check(L.mode_bin.size() == size_t(L.mode_stride), "mode_bin size", ctx);
    int64_t total = 0;
    for (int64_t c : L.bin_count) total += c;
    check(total == lattice, "bin_count total", ctx);
    int64_t with_bin = 0;
    for (int32_t b : L.mode_bin) {
      check(b >= -1 && b < L.n_bins, "mode_bin range", ctx);
      with_bin += b >= 0;
    }
    check(with_bin == L.binned, "mode_bin entries", ctx);
  }
}

void check_layouts() {
  std::vector<int32_t> few = {0, 1, 3, 7};
  std::vector<int32_t> many;
  for (int i = 1; i <= 200; ++i) many.push_back(i);
  std::vector<int32_t> long_lags = {1, 5, 700, 2401, 2500, 2600, 2700, 2800, 2900, 3000, 3100};
  for (int n : {16, 32, 64, 128, 256, 1024}) {
    for (int full = 0; full <= 1; ++full) {
      for (int spec : {NFS_SPEC_F32, NFS_SPEC_BF16, NFS_SPEC_F16}) {
        for (int bwd = 0; bwd <= 1; ++bwd) {
          nfs_desc d = make_desc(n, few, n / 2, 20);
          d.full_spectra = full;
          d.spec_dtype = spec;
          d.backward = bwd;
          d.host_staging = spec == NFS_SPEC_BF16;
          d.accum = spec == NFS_SPEC_F16 ? NFS_ACC_KAHAN : NFS_ACC_PLAIN;
          check_layout(d, 0);
          d.capacity = 0;
          check_layout(d, 0);  // largest lag + 64 slots
          // Derived from the bytes: room for exactly 100 slots after the rest.
          nfs::Layout L0;
          std::string err;
          check(nfs::make_layout(&d, 0, &L0, &err) == NFS_OK, "layout without bytes");
          const size_t slot = size_t(L0.mode_stride) * L0.mode_bytes + nfs::kScaleBytes;
          const size_t bytes = L0.off_ring + 100 * slot + nfs::kAlign;
          check_layout(d, bytes);
          nfs::Layout L1;
          check(nfs::make_layout(&d, bytes, &L1, &err) == NFS_OK && L1.capacity == 100,
                "capacity derived from the bytes");
        }
      }
      nfs_desc d = make_desc(n, many, n / 4 > 0 ? n / 4 : 1, 260);
      d.full_spectra = full;
      check_layout(d, 0);
    }
  }
  for (int n : {16, 64}) {
    nfs_desc d = make_desc(n, long_lags, n / 2, 3200);
    check_layout(d, 0);
    d.accum = NFS_ACC_KAHAN;
    d.full_spectra = 1;
    check_layout(d, 0);
  }
  // n = 4096: only the cheap configuration (the lattice checks are O(n^2)).
  nfs_desc d = make_desc(4096, few, 2048, 10);
  check_layout(d, 0);
}

void check_twiddles() {
  for (int n : {16, 1024, 4096}) {
    const std::vector<float> t = nfs::twiddle_table(n);
    check(t.size() == size_t(2 * n), "twiddle size");
    for (int j = 0; j < n; ++j) {
      const double c = t[size_t(2 * j)], s = t[size_t(2 * j + 1)];
      check(std::fabs(c * c + s * s - 1.0) < 1e-6, "twiddle modulus");
      const double th = 2.0 * 3.14159265358979323846 * j / n;
      check(std::fabs(c - std::cos(th)) < 1e-7 && std::fabs(s + std::sin(th)) < 1e-7,
            "twiddle value");
    }
    check(t[0] == 1.f && t[1] == 0.f && t[size_t(n / 2)] == 0.f && t[size_t(n / 2 + 1)] == -1.f &&
              t[size_t(n)] == -1.f && t[size_t(n + 1)] == 0.f,
          "exact quarter turns");
  }
}

}  // namespace

int main() {
  check_integer_roots();
  check_bins();
  check_validation();
  check_layouts();
  check_twiddles();
  std::printf("all host checks passed (%d checks)\n", g_checks);
  return 0;
}
