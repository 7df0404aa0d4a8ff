// Host-only planning logic; see nfs_host.hpp.
#include "nfs_host.hpp"

#include <algorithm>
#include <cmath>
#include <limits>

namespace nfs {

uint64_t isqrt_u64(uint64_t v) {
  uint64_t s = static_cast<uint64_t>(std::sqrt(static_cast<double>(v)));
  while (s > 0 && s * s > v) --s;
  while ((s + 1) * (s + 1) <= v) ++s;
  return s;
}

int64_t ceil_sqrt_i64(int64_t v) {
  if (v <= 0) return 0;
  int64_t s = static_cast<int64_t>(isqrt_u64(static_cast<uint64_t>(v)));
  return s * s == v ? s : s + 1;
}

int bin_of(int n, int nb, int ky, int kx) {
  const uint64_t r2 = uint64_t(int64_t(kx) * kx + int64_t(ky) * ky);
  const uint64_t b = isqrt_u64(r2 * uint64_t(nb) * uint64_t(nb)) / uint64_t(n / 2);
  return b < uint64_t(nb) ? int(b) : -1;
}

void ring_bounds(int n, int nb, int b, int64_t* lo, int64_t* hi) {
  // |k|^2 nb^2 >= (b m)^2  <=>  |k|^2 >= ceil((b m)^2 / nb^2), m = n/2.
  const int64_t m = n / 2, q = int64_t(nb) * nb;
  const int64_t a = int64_t(b) * m, c = int64_t(b + 1) * m;
  *lo = (a * a + q - 1) / q;
  *hi = (c * c + q - 1) / q;
}

nfs_status validate_desc(const nfs_desc* d, std::string* err) {
  auto fail = [&](nfs_status s, const char* msg) {
    if (err) *err = msg;
    return s;
  };
  if (!d) return fail(NFS_E_ARG, "desc is NULL");
  if (!is_pow2(d->n) || d->n < kMinN || d->n > kMaxN)
    return fail(NFS_E_SIZE, "n must be a power of two in [16, 4096]");
  if (d->in_dtype != NFS_IN_U16 && d->in_dtype != NFS_IN_F32)
    return fail(NFS_E_ARG, "in_dtype must be NFS_IN_U16 or NFS_IN_F32");
  if (d->spec_dtype != NFS_SPEC_F32 && d->spec_dtype != NFS_SPEC_BF16 &&
      d->spec_dtype != NFS_SPEC_F16)
    return fail(NFS_E_UNSUPPORTED, "spec_dtype must be NFS_SPEC_F32, _BF16 or _F16");
  if (d->accum != NFS_ACC_PLAIN && d->accum != NFS_ACC_KAHAN)
    return fail(NFS_E_UNSUPPORTED, "accum must be NFS_ACC_PLAIN or NFS_ACC_KAHAN");
  if (d->host_staging != 0 && d->host_staging != 1)
    return fail(NFS_E_ARG, "host_staging must be 0 or 1");
  if (d->backward != 0 && d->backward != 1) return fail(NFS_E_ARG, "backward must be 0 or 1");
  if (d->full_spectra != 0 && d->full_spectra != 1)
    return fail(NFS_E_ARG, "full_spectra must be 0 or 1");
  if (d->n_lags < 1 || !d->lags) return fail(NFS_E_LAGS, "need at least one lag");
  for (int i = 0; i < d->n_lags; ++i) {
    if (d->lags[i] < 0) return fail(NFS_E_LAGS, "lags must be >= 0");
    if (i && d->lags[i] <= d->lags[i - 1])
      return fail(NFS_E_LAGS, "lags must be strictly increasing");
  }
  if (d->n_bins < 1 || d->n_bins > d->n / 2)
    return fail(NFS_E_BINS, "n_bins must be in [1, n/2]");
  if (d->capacity < 0) return fail(NFS_E_CAPACITY, "capacity must be >= 0");
  if (d->capacity > kMaxCapacity) return fail(NFS_E_CAPACITY, "capacity must be < 2^31");
  if (d->capacity > 0 && d->capacity <= d->lags[d->n_lags - 1])
    return fail(NFS_E_CAPACITY, "capacity must exceed the largest lag");
  return NFS_OK;
}

nfs_status make_layout(const nfs_desc* d, size_t bytes_available, Layout* L,
                       std::string* err) {
  nfs_status st = validate_desc(d, err);
  if (st != NFS_OK) return st;
  Layout& o = *L;
  o = Layout{};
  o.n = d->n;
  o.h = d->n / 2;
  o.n_bins = d->n_bins;
  o.n_lags = d->n_lags;
  o.in_dtype = d->in_dtype;
  o.spec_dtype = d->spec_dtype;
  o.accum = d->accum;
  o.host_staging = d->host_staging;
  o.backward = d->backward;
  o.full = d->full_spectra;
  o.frame_bytes = size_t(d->n) * d->n * (d->in_dtype == NFS_IN_U16 ? 2 : 4);
  o.mode_bytes = d->spec_dtype == NFS_SPEC_F32 ? 8 : 4;
  o.lags.assign(d->lags, d->lags + d->n_lags);
  o.max_lag = o.lags.back();

  // Modes in a ring: k_x in [0, n/2), |k| < n/2; row r has k_y = r
  // (r < n/2) or r - n, and its ring modes are k_x in [0, disc[r]). Plans
  // store those only, or (full) every k_x in [0, n/2] of every row.
  std::vector<int32_t> disc(size_t(o.n));
  const int64_t hh = int64_t(o.h) * o.h;
  int64_t acc = 0;
  for (int r = 0; r < o.n; ++r) {
    const int64_t ky = r < o.h ? r : r - o.n;
    const int64_t rem = hh - 1 - ky * ky;
    const int w = rem < 0 ? 0 : int(isqrt_u64(uint64_t(rem))) + 1;
    disc[size_t(r)] = w;
    acc += w;
  }
  o.binned = acc;
  if (o.full) {
    o.row_width.assign(size_t(o.n), o.h);
    o.modes = int64_t(o.n) * (o.h + 1);
  } else {
    o.row_width = disc;
    o.modes = acc;
  }
  // Slots: tiles of 8 columns, each keeping the rows |k_y| <= R_t with
  // R_t = isqrt((n/2)^2 - 1 - (8t)^2) (the rows where column 8t is stored);
  // full plans keep all n rows of every tile (R_t = n/2) and put the
  // k_x = n/2 column after the tiles, row r in slot nyq_slot + r.
  const int T = o.n / 16;
  o.tiles.assign(size_t(2 * T + 1), 0);
  int64_t base = 0;
  for (int t = 0; t < T; ++t) {
    const int R = o.full ? o.h : int(isqrt_u64(uint64_t(hh - 1 - int64_t(8 * t) * (8 * t))));
    o.tiles[size_t(t)] = int32_t(base);
    o.tiles[size_t(T + 1 + t)] = R;
    base += o.full ? 8 * int64_t(o.n) : 8 * (2 * int64_t(R) + 1);
  }
  o.tiles[size_t(T)] = int32_t(base);
  if (o.full) {
    o.nyq_slot = base;
    base += o.n;
  }
  o.slots = base;
  o.mode_stride = int64_t(align_up(size_t(base), 64));

  // Binning table and segments, rings in order. On row k_y the half-plane
  // modes of ring b are the run k_x in [ceil_sqrt(lo - k_y^2),
  // ceil_sqrt(hi - k_y^2)); every one of them is stored (|k| < n/2).
  o.bin_slots.reserve(size_t(o.binned));
  o.bin_seg0.push_back(0);
  for (int b = 0; b < o.n_bins; ++b) {
    int64_t lo, hi;
    ring_bounds(o.n, o.n_bins, b, &lo, &hi);
    const int R = int(isqrt_u64(uint64_t(hi - 1)));
    const int32_t first = int32_t(o.bin_slots.size());
    for (int ky = -R; ky <= R; ++ky) {
      const int64_t ky2 = int64_t(ky) * ky;
      const int a = lo - ky2 > 0 ? int(ceil_sqrt_i64(lo - ky2)) : 0;
      const int e = int(ceil_sqrt_i64(hi - ky2));
      const int r = ky >= 0 ? ky : ky + o.n;
      for (int kx = a; kx < e; ++kx)
        o.bin_slots.push_back(2 * ring_slot_host(o, r, kx) + (kx > 0 ? 1 : 0));
    }
    const int32_t last = int32_t(o.bin_slots.size());
    int32_t s = first;
    do {
      o.seg_first.push_back(s);
      s += kSegModes;
    } while (s < last);
    o.bin_seg0.push_back(int32_t(o.seg_first.size()));
  }
  o.seg_first.push_back(int32_t(o.bin_slots.size()));
  // The rings partition the modes with |k| < n/2: each is listed exactly once.
  {
    std::vector<char> seen(size_t(o.slots), 0);
    bool ok = int64_t(o.bin_slots.size()) == o.binned;
    for (size_t i = 0; ok && i < o.bin_slots.size(); ++i) {
      const int32_t slot = o.bin_slots[i] >> 1;
      ok = slot >= 0 && slot < o.slots && !seen[size_t(slot)];
      if (ok) seen[size_t(slot)] = 1;
    }
    if (!ok) {
      if (err) *err = "binning table does not list every stored mode once";
      return NFS_E_ARG;
    }
  }

  // Delays up to kMaxLag in LDS-history groups of up to 96, longer ones in
  // groups of up to kGlobalLags for the global-memory kernel.
  int n_short = 0;
  while (n_short < o.n_lags && o.lags[size_t(n_short)] <= kMaxLag) ++n_short;
  const int max_group = kMaxLagsPerWave * kMaxPairWaves;
  for (int first = 0; first < n_short; first += max_group) {
    LagGroup g;
    const int count = std::min(max_group, n_short - first);
    if (!plan_group(o.lags, first, count, &g)) {
      if (err) *err = "lag group does not fit the pair kernel's history";
      return NFS_E_LAGS;
    }
    o.groups.push_back(g);
  }
  for (int first = n_short; first < o.n_lags; first += kGlobalLags) {
    LagGroup g;
    g.first = first;
    g.count = std::min(kGlobalLags, o.n_lags - first);
    g.max_lag = o.lags[size_t(first + g.count - 1)];
    g.modes = 0;
    o.groups.push_back(g);
  }

  const size_t inter_frame = size_t(o.n) * o.h * 8;
  o.batch = int(std::max<size_t>(1, std::min<size_t>(kMaxBatch, kBatchBytes / inter_frame)));
  // A batch never exceeds what the ring can take beyond the largest lag.
  if (d->capacity > 0) o.batch = int(std::min<int64_t>(o.batch, d->capacity - o.max_lag));

  // Everything except the ring.
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t at = off;
    off = align_up(off + bytes, kAlign);
    return at;
  };
  o.off_inter = take(size_t(o.batch) * inter_frame);
  o.off_rowsum = take(size_t(o.batch) * o.n * 8);
  // Row sums of |frame - reference|, for the FP16 scale only.
  o.off_rowabs = take(o.spec_dtype == NFS_SPEC_F16 ? size_t(o.batch) * o.n * 8 : 0);
  o.off_nyq = take(o.full ? size_t(o.batch) * o.n * 4 : 0);
  o.off_acc = take(size_t(o.n_lags) * o.mode_stride * 4);
  o.off_comp = take(o.accum == NFS_ACC_KAHAN ? size_t(o.n_lags) * o.mode_stride * 4 : 0);
  // Fused transform at n = 1024: per launch at most `batch` jobs; its
  // buffers (8 XCDs x 4 MiB) fit the intermediate from 8 frames on.
  o.fused_ok = o.n == 1024 && !o.full && size_t(o.batch) * inter_frame >= (size_t(32) << 20);
  o.fused_slots = (o.batch + 7) / 8;  // frames per XCD per launch at most
  o.off_sched = take(o.fused_ok ? size_t(8 * 64 + 16 * o.fused_slots) * 4 : 0);
  const size_t nseg = o.seg_first.size() - 1;
  o.off_segs = take((o.seg_first.size() + o.bin_seg0.size()) * 4);
  o.off_bin_slots = take(o.bin_slots.size() * 4);
  o.off_part = take(nseg * o.n_lags * 8);
  o.off_part_cnt = take(nseg * 8);
  o.off_status = take(kAlign);
  o.off_tw = take(size_t(o.n) * 8);
  o.off_width = take(size_t(o.n) * 4);
  o.off_tiles = take(o.tiles.size() * 4);
  o.off_lags = take(size_t(o.n_lags) * 4);
  o.off_ref = take(o.frame_bytes);
  o.off_stage = take(o.host_staging ? 2 * size_t(o.batch) * o.frame_bytes : 0);
  if (o.backward) {
    // k-space gradients of a batch, later its g' images (n x n floats).
    o.off_gk = take(size_t(o.batch) * std::max(size_t(o.mode_stride) * 8, size_t(o.n) * o.n * 4));
    o.off_brow = take(size_t(o.batch) * o.n * 16);
    o.off_bscal = take(size_t(o.batch) * 16);
    o.off_gw = take(size_t(o.n) * o.n * 8);
    o.off_gtab = take(size_t(o.n_lags) * o.n_bins * 4);
    o.off_mode_bin = take(size_t(o.mode_stride) * 4);
    o.off_bin_count = take(size_t(o.n_bins) * 8);
    // Bin of every stored mode and C_b, the full-plane modes of each bin:
    // a half-plane mode with k_x > 0 stands for itself and its mirror.
    // Slots of modes that are not stored get -1 (no gradient).
    o.mode_bin.assign(size_t(o.mode_stride), -1);
    o.bin_count.assign(size_t(o.n_bins), 0);
    const uint64_t nb2 = uint64_t(o.n_bins) * uint64_t(o.n_bins);
    for (int r = 0; r < o.n; ++r) {
      const int64_t ky = r < o.h ? r : r - o.n;
      for (int kx = 0; kx < disc[size_t(r)]; ++kx) {
        const uint64_t k2 = uint64_t(ky * ky) + uint64_t(kx) * uint64_t(kx);
        const int b = int(isqrt_u64(k2 * nb2) / uint64_t(o.h));
        o.mode_bin[size_t(ring_slot_host(o, r, kx))] = b;
        o.bin_count[size_t(b)] += kx == 0 ? 1 : 2;
      }
    }
  }
  o.off_refspec = take(size_t(o.mode_stride) * 8);
  o.off_ring = off;
  // Each ring slot holds one spectrum (8 or 4 bytes per mode, whole
  // multiples of kAlign bytes) and, after the ring, its frame's scales.
  const size_t spec_bytes = size_t(o.mode_stride) * o.mode_bytes;
  const size_t slot_bytes = spec_bytes + kScaleBytes;

  if (d->capacity > 0) {
    o.capacity = d->capacity;
  } else if (bytes_available > 0) {
    if (bytes_available <= o.off_ring + kAlign) {
      if (err) *err = "workspace too small for any spectrum ring";
      return NFS_E_WORKSPACE;
    }
    o.capacity = std::min<int64_t>(kMaxCapacity,
                                   int64_t((bytes_available - o.off_ring - kAlign) / slot_bytes));
  } else {
    o.capacity = int64_t(o.max_lag) + 64;
  }
  if (o.capacity <= o.max_lag) {
    if (err) *err = "ring capacity must exceed the largest lag";
    return NFS_E_CAPACITY;
  }
  o.off_fscale = o.off_ring + size_t(o.capacity) * spec_bytes;
  o.total = align_up(o.off_fscale + size_t(o.capacity) * kScaleBytes, kAlign);
  return NFS_OK;
}

int ring_slot_host(const Layout& L, int r, int kx) {
  const int T = L.n / 16;
  const int t = kx / 8;
  const int R = L.tiles[size_t(T + 1 + t)];
  if (R >= L.h) return L.tiles[size_t(t)] + r * 8 + kx % 8;
  const int ky = r < L.h ? r : r - L.n;
  if (ky > R || -ky > R) return -1;
  const int rank = r <= R ? r : r - (L.n - 2 * R - 1);
  return L.tiles[size_t(t)] + rank * 8 + kx % 8;
}

std::vector<float> twiddle_table(int n) {
  // theta = 2 pi j / n = q * (pi/2) + phi with q the quadrant; cos and sin of
  // phi in [0, pi/2) in double, rotated by q quarter turns exactly, so the
  // table is exact at multiples of pi/2 and symmetric between quadrants.
  std::vector<float> t(size_t(2) * n);
  const double half_pi = 1.5707963267948966192313216916398;
  for (int j = 0; j < n; ++j) {
    const int64_t j4 = int64_t(4) * j;
    const int q = int(j4 / n);
    const int64_t rem = j4 - int64_t(q) * n;
    const double phi = half_pi * double(rem) / double(n);
    const double c0 = rem ? std::cos(phi) : 1.0;
    const double s0 = rem ? std::sin(phi) : 0.0;
    double c = c0, s = s0;
    if (q == 1) { c = -s0; s = c0; }
    if (q == 2) { c = -c0; s = -s0; }
    if (q == 3) { c = s0; s = -c0; }
    t[2 * j] = float(c);
    t[2 * j + 1] = float(-s);
  }
  return t;
}

}  // namespace nfs
