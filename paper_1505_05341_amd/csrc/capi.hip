// C interface of libpk: configuration checks, the workspace plan and the sequence of
// stages on the caller's stream (declared in include/pk.h).
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <mutex>
#include <string>
#include <vector>

#include "basis.hpp"
#include "plan.hpp"

namespace pk {

static thread_local std::string g_last_error;

static pk_status fail(pk_status st, const std::string& why) {
  g_last_error = why;
  return st;
}

static int num_grids_for(int ell) { return ell == 0 ? 1 : (ell == 2 ? 7 : (ell == 4 ? 22 : 50)); }
static bool ell_ok(int ell) { return ell == 0 || ell == 2 || ell == 4 || ell == 6; }

static int64_t isqrt64(int64_t n) {
  if (n <= 0) return 0;
  int64_t s = (int64_t)sqrt((double)n);
  while (s * s > n) --s;
  while ((s + 1) * (s + 1) <= n) ++s;
  return s;
}

static size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

// Device result layout (doubles): k_eff[nb], P[nl][nb], noise[nb], nmodes[nb],
// wedges[2][nb], then alpha, I, S and the error flags.
static int64_t result_size(int nb, int nl) { return (int64_t)nb * (5 + nl) + 4; }


static bool supported_N(int N) {
  return N == 8 || N == 16 || N == 32 || N == 64 || N == 128 || N == 256 || N == 512 || N == 1024 || N == 2048;
}

// Automatic slab: all planes while the x-transformed grids take at most 128 GiB (every N
// up to 1024), else the largest power of two of planes whose two slots fit in 8 GiB.
static int auto_slab(int N, int G, int Kx) {
  if (8.0 * G * (double)N * Kx * N <= 128.0 * (1ull << 30)) return N;
  const double plane = 8.0 * G * (double)N * Kx;
  int xs = N;
  while (xs > 1 && 2.0 * plane * xs > 8.0 * (1ull << 30)) xs >>= 1;
  return xs;
}

// Schedules of the column transforms (values per thread of the y and z passes), per
// (N, ell_max): set by pk_set_schedule or the autotuner; 0 = not set, meaning 8 for both:
// the y pass then sums up to 6 z-power groups at once (with 16 values only 3 fit its
// registers, so grids shared by more groups are loaded more than once), and the z pass's
// prefetched column does not fit the registers of the 16-value schedule.
struct Schedule {
  int y, z;
};
static Schedule g_sched[12][4];

static int log2_of(int N) {
  int l = 0;
  while ((1 << l) < N) ++l;
  return l;
}

// Groups (n, c) and their members (grid index, a, b, multinomial weight n!/(a! b! c!)).
static void build_groups(int ell, GroupTable* gt) {
  static const int fact[7] = {1, 1, 2, 6, 24, 120, 720};
  gt->ngroups = 0;
  for (int n = 0; n <= ell; n += 2) {
    for (int c = 0; c <= n; ++c) {
      const int g = gt->ngroups++;
      gt->n[g] = n;
      gt->c[g] = c;
      gt->count[g] = 0;
      for (int m = 0; m < num_grids_for(ell); ++m) {
        const Monomial mo = monomial(m);
        if (mo.a + mo.b + mo.c != n || mo.c != c) continue;
        const int s = gt->count[g]++;
        gt->grid[g][s] = m;
        gt->a[g][s] = mo.a;
        gt->b[g][s] = mo.b;
        gt->coef[g][s] = (float)(fact[n] / (fact[mo.a] * fact[mo.b] * fact[mo.c]));
      }
    }
  }
}

// Sets of the y pass (see YSetTable) for groups of at most gmax: the groups of each parity
// of c in order, gmax at a time; a set's members are the gathered grids, in gathered order,
// that carry a term of one of its groups. A member (a, b, c) of group (n, c) with weight
// coef contributes coef w tx^a ty^b to gathered grid j, w the integer weight of j in the
// identity's expansion of rhat^(a,b,c) (basis.hpp; 1 if (a, b, c) is gathered itself).
// At most 6 sets, 56 members and 119 terms (ell_max = 6 with sets of 3): within the
// table's bounds for every ell_max.
static void build_ysets(const GroupTable& gt, int ell, int gmax, YSetTable* yt) {
  memset(yt, 0, sizeof(*yt));
  const int GK = kept_count(ell), ND = dep_count(ell);
  int kidx[kMaxGrids], didx[kMaxGrids];
  for (int m = 0; m < kMaxGrids; ++m) kidx[m] = didx[m] = -1;
  for (int j = 0; j < GK; ++j) kidx[kept_monomial(j)] = j;
  for (int d = 0; d < ND; ++d) didx[dep_monomial(d)] = d;
  int nm = 0, nt = 0;
  for (int par = 0; par < 2; ++par) {
    int gs[kMaxGroups], ng = 0;
    for (int g = 0; g < gt.ngroups; ++g)
      if (gt.c[g] % 2 == par) gs[ng++] = g;
    for (int i0 = 0; i0 < ng; i0 += gmax) {
      const int s = yt->nsets++;
      const int k = ng - i0 < gmax ? ng - i0 : gmax;
      yt->ngroups[s] = (int8_t)k;
      for (int q = 0; q < k; ++q) yt->group[s][q] = (int8_t)gs[i0 + q];
      yt->mem0[s] = (int16_t)nm;
      for (int j = 0; j < GK; ++j) {
        const int t0 = nt;
        for (int q = 0; q < k; ++q) {
          const int g = gs[i0 + q];
          for (int u = 0; u < gt.count[g]; ++u) {
            const int m = gt.grid[g][u];
            int w = 0;
            if (kidx[m] >= 0) {
              w = kidx[m] == j ? 1 : 0;
            } else {
              const int d = didx[m];
              for (int v = 0; v < dep_terms(d); ++v)
                if (dep_kept(d, v) == j) w += (int)dep_coef(d, v);
            }
            if (w == 0) continue;
            yt->tslot[nt] = (int8_t)q;
            yt->ta[nt] = (int8_t)gt.a[g][u];
            yt->tb[nt] = (int8_t)gt.b[g][u];
            yt->tcoef[nt] = gt.coef[g][u] * (float)w;
            ++nt;
          }
        }
        if (nt > t0) {
          yt->mgrid[nm] = (int8_t)j;
          yt->term0[nm] = (int16_t)t0;
          ++nm;
        }
      }
    }
  }
  yt->mem0[yt->nsets] = (int16_t)nm;
  yt->term0[nm] = (int16_t)nt;
}

pk_status make_plan(const pk_config* cfg, int64_t n_gal, int64_t n_ran, Plan* plan, const char** why) {
  static const char* msg = "";
  *why = msg;
  if (!cfg) return fail(PK_EINVAL, "null configuration");
  Plan& p = *plan;
  memset(&p, 0, sizeof(Plan));
  p.N = cfg->N;
  p.assign = cfg->assign;
  p.ell_max = cfg->ell_max;
  p.los = cfg->los;
  p.compensate = cfg->compensate;
  p.dn = cfg->dn;
  p.nbins = cfg->nbins;
  p.norm_from = cfg->norm_from;
  for (int i = 0; i < 3; ++i) {
    p.box_min[i] = cfg->box_min[i];
    p.observer[i] = cfg->observer[i];
  }
  p.L = cfg->L;
  p.n_gal = n_gal;
  p.n_ran = n_ran;
  if (!supported_N(p.N)) return fail(PK_ENOTSUP, "N must be one of 8, 16, 32, 64, 128, 256, 512, 1024, 2048");
  if (p.assign != PK_CIC && p.assign != PK_TSC) return fail(PK_EINVAL, "assign must be 2 (CIC) or 3 (TSC)");
  if (!ell_ok(p.ell_max)) return fail(PK_EINVAL, "ell_max must be 0, 2, 4 or 6");
  if (p.los != 0 && p.los != 1) return fail(PK_EINVAL, "los must be 0 or 1");
  if (p.compensate < 0 || p.compensate > 2) return fail(PK_EINVAL, "compensate must be 0, 1 or 2");
  if (p.norm_from != 0 && p.norm_from != 1) return fail(PK_EINVAL, "norm_from must be 0 or 1");
  if (p.dn < 1) return fail(PK_EINVAL, "dn must be >= 1");
  if (p.nbins < 1 || (int64_t)p.nbins * p.dn > p.N / 2) return fail(PK_EINVAL, "need 1 <= nbins and nbins * dn <= N / 2");
  if (!(p.L > 0.0) || !isfinite(p.L)) return fail(PK_EINVAL, "L must be positive and finite");
  for (int i = 0; i < 3; ++i)
    if (!isfinite(p.box_min[i]) || !isfinite(p.observer[i])) return fail(PK_EINVAL, "box_min and observer must be finite");
  if (n_gal < 0 || n_ran < 0) return fail(PK_EINVAL, "catalogue sizes must be >= 0");
  if (n_gal + n_ran > (int64_t)0x7fffffff) return fail(PK_ENOTSUP, "at most 2^31 - 1 particles per call");
  if (p.ell_max == 6 && p.N > 1024) return fail(PK_ENOTSUP, "ell_max = 6 is built for N <= 1024");
  if (cfg->x_planes < 0 || cfg->x_planes > p.N || (cfg->x_planes & (cfg->x_planes - 1)) != 0)
    return fail(PK_EINVAL, "x_planes must be 0 (automatic) or a power of two <= N");

  p.G = num_grids_for(p.ell_max);
  p.GK = kept_count(p.ell_max);
  p.K = p.nbins * p.dn;
  p.TK = p.N >= 2048 ? 4 : (p.N >= 1024 ? 8 : (p.N / 2 < 16 ? p.N / 2 : 16));  // tile_cols<N>() of the FFT passes
  p.Kx = ((p.K + p.TK - 1) / p.TK) * p.TK;
  p.nkt = p.Kx / p.TK;
  p.xs = cfg->x_planes ? cfg->x_planes : auto_slab(p.N, p.GK, p.Kx);
  p.xr = p.N / p.xs < 2 ? 1 : 2;  // X holds two slabs (double buffer) when there are several
  // tiles: the y pass keeps |ky| <= M(kt) with kx0^2 + ky^2 < K^2, kx0 = kt * TK
  int64_t reg = 0, items = 0;
  for (int kt = 0; kt < p.nkt; ++kt) {
    const int64_t kx0 = (int64_t)kt * p.TK;
    const int64_t M = isqrt64((int64_t)p.K * p.K - 1 - kx0 * kx0);
    p.tiles.M[kt] = (int)M;
    p.tiles.regoff[kt] = reg;
    p.tiles.item0[kt] = items;
    reg += (int64_t)p.N * (2 * M + 1) * p.TK;
    items += 2 * M + 1;
  }
  p.tiles.item0[p.nkt] = items;
  p.H_group_stride = (size_t)reg;
  p.z_items = items;
  p.z_blocks = (int)(items < 512 ? items : 512);
  const Schedule sc = g_sched[log2_of(p.N)][p.ell_max / 2];
  p.col_e[0] = p.N >= 2048 ? 8 : (sc.y ? sc.y : 8);  // only the 8-value schedule is built at 2048
  p.col_e[1] = p.N >= 2048 ? 8 : (sc.z ? sc.z : 8);

  GroupTable& gt = p.groups;
  build_groups(p.ell_max, &gt);
  build_ysets(gt, p.ell_max, kYSetGroups, &p.ysets[0]);
  build_ysets(gt, p.ell_max, 3, &p.ysets[1]);

  const int nl = p.ell_max / 2 + 1;
  p.result_doubles = result_size(p.nbins, nl);
  const int64_t nrow = (int64_t)p.N * p.N;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off = align256(off + bytes);
    return o;
  };
  p.off_scalars = take(sizeof(double) * 16);
  p.off_partials = take(sizeof(double) * 6 * kStatsBlocks);
  p.off_flags = take(64);
  p.off_tw = take(sizeof(float) * 2 * p.N);
  p.off_invw2 = take(sizeof(float) * p.N);
  p.off_alias = take(sizeof(float) * p.N);
  p.off_tables = take(tables_bytes());
  p.off_rowcnt = take(sizeof(uint32_t) * ((size_t)p.N * sort_blocks(n_gal + n_ran) + 1));  // plane histograms
  p.off_rowoff = take(sizeof(uint32_t) * (nrow + 1));
  p.off_rowhist = take(sizeof(uint32_t) * ((size_t)nrow * kRowHistParts + 1));  // per-part row counts
  p.off_blocksum = take(sizeof(uint32_t) * kScanTopMax);
  p.off_tmp = take(sizeof(float) * 4 * (size_t)(n_gal + n_ran));
  p.off_rowkey = take(sizeof(uint16_t) * (size_t)(n_gal + n_ran));
  p.off_sorted = take(sizeof(float) * 4 * (size_t)(n_gal + n_ran));
  p.off_X = take(sizeof(float) * 2 * (size_t)p.GK * p.xr * p.xs * p.N * p.Kx);  // xr slots of xs planes
  p.off_H = take(sizeof(float) * 2 * (size_t)gt.ngroups * p.H_group_stride);
  p.off_zpart = take(sizeof(double) * kNumSums * (size_t)p.z_blocks * p.nbins);
  p.off_result = take(sizeof(double) * (size_t)p.result_doubles);
  p.total = off;
  return PK_OK;
}

static pk_status check_catalog(const pk_catalog* c, bool need_nbar, const char* name) {
  if (!c) return fail(PK_EINVAL, std::string("null ") + name + " catalogue");
  if (c->n < 0) return fail(PK_EINVAL, std::string(name) + ".n < 0");
  if (c->n > 0 && (!c->xyz || !c->w)) return fail(PK_EINVAL, std::string(name) + ": null xyz or w");
  if (c->n > 0 && need_nbar && !c->nbar) return fail(PK_EINVAL, std::string(name) + ": nbar is needed by the normalisation");
  return PK_OK;
}

static pk_status hip_fail(hipError_t e, const char* where) {
  return fail(PK_EDEVICE, std::string(where) + ": " + hipGetErrorString(e));
}

static pk_status prepare_plan(const pk_config* cfg, const pk_catalog* gal, const pk_catalog* ran, Plan* p) {
  pk_status st = check_catalog(gal, cfg && cfg->norm_from == 1, "galaxy");
  if (st != PK_OK) return st;
  st = check_catalog(ran, cfg && cfg->norm_from == 0, "random");
  if (st != PK_OK) return st;
  const char* why;
  return make_plan(cfg, gal->n, ran->n, p, &why);
}

static pk_status prepare(const pk_config* cfg, const pk_catalog* gal, const pk_catalog* ran, void* ws,
                         size_t ws_bytes, Plan* p) {
  const pk_status st = prepare_plan(cfg, gal, ran, p);
  if (st != PK_OK) return st;
  if (!ws || ws_bytes < p->total)
    return fail(PK_EWORKSPACE, "workspace needs " + std::to_string(p->total) + " bytes, got " + std::to_string(ws_bytes));
  if (((uintptr_t)ws & 255) != 0) return fail(PK_EWORKSPACE, "workspace must be 256-byte aligned");
  return PK_OK;
}

// Stage timing (measurement only): events recorded between the stages of a call.
constexpr int kNumStages = 7;
static const char* kStageNames[kNumStages] = {"init", "scalars", "sort", "assign_x", "fft_y", "fft_z_bin",
                                               "finalize"};
static struct {
  bool enabled = false;
  bool recorded = false;
  int device = -1;
  hipEvent_t ev[kNumStages + 1] = {};
} g_timing;

static void mark(int i, hipStream_t s) {
  if (g_timing.enabled && g_timing.ev[i]) hipEventRecord(g_timing.ev[i], s);
}

// Second stream of the calling thread on each device, on which the y pass of slab i runs
// while the x pass of slab i + 1 runs on the caller's stream (the x pass is bound by
// arithmetic, the y pass by memory). Default priority, non-blocking; events order the
// two: y(i) after x(i), and with two slots x(i) after y(i - 2).
constexpr int kMaxDevices = 16;
constexpr int kPipeEvents = 64;
struct Pipe {
  bool ready = false;
  hipStream_t aux = nullptr;
  hipEvent_t fork = nullptr, ex[kPipeEvents] = {}, ey[kPipeEvents] = {};
};
static thread_local Pipe g_pipe[kMaxDevices];

static hipError_t pipe_for_device(Pipe** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  Pipe& pp = g_pipe[dev];
  if (!pp.ready) {
    if ((e = hipStreamCreateWithFlags(&pp.aux, hipStreamNonBlocking)) != hipSuccess) return e;
    if ((e = hipEventCreateWithFlags(&pp.fork, hipEventDisableTiming)) != hipSuccess) return e;
    for (int i = 0; i < kPipeEvents; ++i) {
      if ((e = hipEventCreateWithFlags(&pp.ex[i], hipEventDisableTiming)) != hipSuccess) return e;
      if ((e = hipEventCreateWithFlags(&pp.ey[i], hipEventDisableTiming)) != hipSuccess) return e;
    }
    pp.ready = true;
  }
  *out = &pp;
  return hipSuccess;
}

// The x and y passes over every slab. Slab i covers planes [i xs, (i + 1) xs) and uses
// slot i mod xr of X. With one slab, or while `s` is being captured into a graph, both
// passes run in order on `s`; otherwise the y passes run on the second stream, each after
// its slab's x pass (an event on `s`), and an x pass that reuses a slot waits for the y
// pass that read it; `s` finally waits for the last y pass.
static hipError_t run_slabs(const Plan& p, char* ws, hipStream_t s, bool stop_after_x, bool timed, bool one_stream) {
  const int nslab = p.N / p.xs;
  hipError_t e;
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  if ((e = hipStreamIsCapturing(s, &cs)) != hipSuccess) return e;
  Pipe* pp = nullptr;
  if (nslab > 1 && !stop_after_x && !one_stream && cs == hipStreamCaptureStatusNone && p.xr <= kPipeEvents) {
    if ((e = pipe_for_device(&pp)) != hipSuccess) return e;
  }
  if (!pp) {
    for (int i = 0; i < nslab; ++i) {
      const int z0 = i * p.xs, pb = (i % p.xr) * p.xs;
      if ((e = launch_xpass(p, ws, s, z0, pb)) != hipSuccess) return e;
      if (stop_after_x) return hipSuccess;  // X holds the first slab
      if (timed && nslab == 1) mark(4, s);
      if ((e = launch_ypass(p, ws, s, z0, pb)) != hipSuccess) return e;
    }
    return hipSuccess;
  }
  if ((e = hipEventRecord(pp->fork, s)) != hipSuccess) return e;
  if ((e = hipStreamWaitEvent(pp->aux, pp->fork, 0)) != hipSuccess) return e;
  for (int i = 0; i < nslab; ++i) {
    const int z0 = i * p.xs, pb = (i % p.xr) * p.xs;
    if (i >= p.xr && (e = hipStreamWaitEvent(s, pp->ey[(i - p.xr) % kPipeEvents], 0)) != hipSuccess) return e;
    if ((e = launch_xpass(p, ws, s, z0, pb)) != hipSuccess) return e;
    if ((e = hipEventRecord(pp->ex[i % kPipeEvents], s)) != hipSuccess) return e;
    if ((e = hipStreamWaitEvent(pp->aux, pp->ex[i % kPipeEvents], 0)) != hipSuccess) return e;
    if ((e = launch_ypass(p, ws, pp->aux, z0, pb)) != hipSuccess) return e;
    if ((e = hipEventRecord(pp->ey[i % kPipeEvents], pp->aux)) != hipSuccess) return e;
  }
  return hipStreamWaitEvent(s, pp->ey[(nslab - 1) % kPipeEvents], 0);
}

// Where a call stops: after the x transforms of the first slab (X left in the workspace),
// after the y transforms of every slab (H left in the workspace), or at the end.
enum class Stop { kAfterX, kAfterY, kNone };

static pk_status run_stages(const Plan& p, const pk_catalog& gal, const pk_catalog& ran, char* ws, double* d_result,
                            hipStream_t s, Stop stop, bool one_stream = false) {
  hipError_t e;
  const bool stop_after_x = stop == Stop::kAfterX;
  const bool timed = g_timing.enabled && stop == Stop::kNone && !one_stream;
  if (timed) {
    int dev = -1;
    hipGetDevice(&dev);
    if (g_timing.device != dev) {
      for (int i = 0; i <= kNumStages; ++i)
        if (hipEventCreate(&g_timing.ev[i]) != hipSuccess) g_timing.ev[i] = nullptr;
      g_timing.device = dev;
    }
    g_timing.recorded = false;
  }
  if (timed) mark(0, s);
  if ((e = launch_init(p, ws, s)) != hipSuccess) return hip_fail(e, "init");
  if (timed) mark(1, s);
  if ((e = launch_stats(p, gal, ran, ws, s)) != hipSuccess) return hip_fail(e, "catalogue scalars");
  if (timed) mark(2, s);
  if ((e = launch_sort(p, gal, ran, ws, s)) != hipSuccess) return hip_fail(e, "row sort");
  if (timed) mark(3, s);
  // with one slab (xs = N) the x and y stages are timed apart; with several, "assign_x"
  // covers both
  if ((e = run_slabs(p, ws, s, stop_after_x, timed, one_stream)) != hipSuccess)
    return hip_fail(e, "x and y transforms");
  if (stop != Stop::kNone) return PK_OK;
  if (timed && p.xs != p.N) mark(4, s);
  if (timed) mark(5, s);
  if ((e = launch_zpass(p, ws, s)) != hipSuccess) return hip_fail(e, "z transform and binning");
  if (timed) mark(6, s);
  if ((e = launch_finalize(p, ws, d_result, s)) != hipSuccess) return hip_fail(e, "finalize");
  if (timed) {
    mark(7, s);
    g_timing.recorded = true;
  }
  return PK_OK;
}

// Copies the device result of a call to the caller's host arrays (waits for the stream).
static pk_status fetch_result(const Plan& p, const double* d_res, hipStream_t s, pk_result* out);

static pk_status flags_status(int flags);

static pk_status unpack_result(const double* r, int nb, int nl, pk_result* o) {
  const double* tail = r + (size_t)nb * (5 + nl);
  const pk_status st = flags_status((int)tail[3]);
  if (st != PK_OK) return st;
  if (o->k_eff) memcpy(o->k_eff, r, sizeof(double) * nb);
  if (o->P) memcpy(o->P, r + nb, sizeof(double) * nb * nl);
  if (o->noise) memcpy(o->noise, r + (size_t)nb * (1 + nl), sizeof(double) * nb);
  if (o->nmodes)
    for (int b = 0; b < nb; ++b) o->nmodes[b] = (int64_t)r[(size_t)nb * (2 + nl) + b];
  if (o->wedges) memcpy(o->wedges, r + (size_t)nb * (3 + nl), sizeof(double) * 2 * nb);
  o->alpha = tail[0];
  o->I = tail[1];
  o->S = tail[2];
  return PK_OK;
}

static pk_status fetch_result(const Plan& p, const double* d_res, hipStream_t s, pk_result* out) {
  std::vector<double> h((size_t)p.result_doubles);
  hipError_t e = hipMemcpyAsync(h.data(), d_res, sizeof(double) * h.size(), hipMemcpyDeviceToHost, s);
  if (e != hipSuccess) return hip_fail(e, "result copy");
  e = hipStreamSynchronize(s);
  if (e != hipSuccess) return hip_fail(e, "stream synchronize");
  return unpack_result(h.data(), p.nbins, p.ell_max / 2 + 1, out);
}

static pk_status flags_status(int flags) {
  if (flags & kFlagOutOfBox) return fail(PK_ERANGE, "a particle lies outside [box_min, box_min + L)");
  if (flags & kFlagNonFinitePos) return fail(PK_EDOM, "a particle position is not finite");
  if (flags & kFlagAtObserver) return fail(PK_EDOM, "a particle sits at the observer (no line of sight)");
  if (flags & kFlagNonFiniteWeight) return fail(PK_EDOM, "a weight or nbar is not finite");
  if (flags & kFlagBadNorm) return fail(PK_EDOM, "sum of random weights is 0 or the normalisation I is not positive");
  return PK_OK;
}

}  // namespace pk

using namespace pk;

extern "C" {

pk_status pk_workspace_size(const pk_config* cfg, int64_t n_gal, int64_t n_ran, size_t* bytes) {
  if (!bytes) return fail(PK_EINVAL, "null bytes pointer");
  Plan p;
  const char* why;
  const pk_status st = make_plan(cfg, n_gal, n_ran, &p, &why);
  if (st != PK_OK) return st;
  *bytes = p.total;
  return PK_OK;
}

int64_t pk_result_doubles(const pk_config* cfg) {
  if (!cfg || !ell_ok(cfg->ell_max) || cfg->nbins < 1) return -1;
  return result_size(cfg->nbins, cfg->ell_max / 2 + 1);
}

pk_status pk_multipoles_async(const pk_config* cfg, const pk_catalog* gal, const pk_catalog* ran, void* workspace,
                              size_t workspace_bytes, double* d_result, void* hip_stream) {
  Plan p;
  pk_status st = prepare(cfg, gal, ran, workspace, workspace_bytes, &p);
  if (st != PK_OK) return st;
  if (!d_result) return fail(PK_EINVAL, "null result pointer");
  return run_stages(p, *gal, *ran, static_cast<char*>(workspace), d_result, (hipStream_t)hip_stream, Stop::kNone);
}

pk_status pk_multipoles(const pk_config* cfg, const pk_catalog* gal, const pk_catalog* ran, void* workspace,
                        size_t workspace_bytes, pk_result* out, void* hip_stream) {
  Plan p;
  pk_status st = prepare(cfg, gal, ran, workspace, workspace_bytes, &p);
  if (st != PK_OK) return st;
  if (!out) return fail(PK_EINVAL, "null result");
  char* ws = static_cast<char*>(workspace);
  hipStream_t s = (hipStream_t)hip_stream;
  double* d_res = at<double>(ws, p.off_result);
  st = run_stages(p, *gal, *ran, ws, d_res, s, Stop::kNone);
  if (st != PK_OK) return st;
  return fetch_result(p, d_res, s, out);
}

// --------------------------------------------------- entry point that allocates nothing
// For callers that cannot allocate (code being captured into a graph, serving loops,
// harnesses that forbid allocation): the workspace is a fixed array in the library's
// device image. Each GPU holds its own copy of it from the first launch of any of the
// library's kernels until the process ends. In host code the array's name is only a
// stand-in; its device address, which differs per GPU, is taken once per device with
// hipGetSymbolAddress and used everywhere instead of the name.
constexpr size_t kScratchBytes = PK_NOALLOC_SCRATCH_BYTES;
constexpr int kScratchResultMax = 1024;  // doubles of the result staging buffer
static __device__ __align__(256) char scratch[kScratchBytes];
static std::mutex g_scratch_mu;
static char* g_scratch_dev[kMaxDevices];

static pk_status scratch_for_device(char** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "get device");
  if (dev < 0 || dev >= kMaxDevices) return fail(PK_EDEVICE, "device index beyond the library's per-device table");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_dev[dev]) {
    void* ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return hip_fail(e, "address of the scratch array");
    if (!ptr || ((uintptr_t)ptr & 255) != 0) return fail(PK_EDEVICE, "scratch array missing or misaligned");
    g_scratch_dev[dev] = static_cast<char*>(ptr);
  }
  *out = g_scratch_dev[dev];
  return PK_OK;
}

pk_status pk_multipoles_noalloc(const pk_config* cfg, const pk_catalog* gal, const pk_catalog* ran, pk_result* out,
                                void* hip_stream) {
  Plan p;
  pk_status st = prepare_plan(cfg, gal, ran, &p);
  if (st != PK_OK) return st;
  if (!out) return fail(PK_EINVAL, "null result");
  if (p.total > kScratchBytes)
    return fail(PK_EWORKSPACE, "this configuration needs " + std::to_string(p.total) +
                                   " bytes of scratch; pk_multipoles_noalloc holds " +
                                   std::to_string(kScratchBytes) + " (use pk_multipoles with a workspace)");
  if (p.result_doubles > kScratchResultMax)
    return fail(PK_EWORKSPACE, "too many bins for pk_multipoles_noalloc's result buffer");
  char* ws = nullptr;
  if ((st = scratch_for_device(&ws)) != PK_OK) return st;
  hipStream_t s = (hipStream_t)hip_stream;
  double* d_res = at<double>(ws, p.off_result);
  // one stream only (no second stream for slabs) and no timing events: nothing is created
  st = run_stages(p, *gal, *ran, ws, d_res, s, Stop::kNone, /*one_stream=*/true);
  if (st != PK_OK) return st;
  static thread_local double h[kScratchResultMax];
  hipError_t e = hipMemcpyAsync(h, d_res, sizeof(double) * (size_t)p.result_doubles, hipMemcpyDeviceToHost, s);
  if (e != hipSuccess) return hip_fail(e, "result copy");
  if ((e = hipStreamSynchronize(s)) != hipSuccess) return hip_fail(e, "stream synchronize");
  return unpack_result(h, p.nbins, p.ell_max / 2 + 1, out);
}

// ------------------------------------------------------------------- FFT schedules

static bool schedule_key_ok(int32_t N, int32_t ell_max) {
  return supported_N(N) && ell_ok(ell_max);
}

pk_status pk_set_schedule(int32_t N, int32_t ell_max, int32_t y_values, int32_t z_values) {
  if (!schedule_key_ok(N, ell_max)) return fail(PK_EINVAL, "unsupported N or ell_max");
  if ((y_values != 8 && y_values != 16) || (z_values != 8 && z_values != 16))
    return fail(PK_EINVAL, "values per thread must be 8 or 16");
  if (N >= 2048 && (y_values != 8 || z_values != 8))
    return fail(PK_EINVAL, "at N = 2048 only the 8-value schedule is built");
  g_sched[log2_of(N)][ell_max / 2] = Schedule{y_values, z_values};
  return PK_OK;
}

pk_status pk_get_schedule(int32_t N, int32_t ell_max, int32_t* y_values, int32_t* z_values) {
  if (!schedule_key_ok(N, ell_max)) return fail(PK_EINVAL, "unsupported N or ell_max");
  if (!y_values || !z_values) return fail(PK_EINVAL, "null output pointer");
  const Schedule sc = g_sched[log2_of(N)][ell_max / 2];
  *y_values = N >= 2048 ? 8 : (sc.y ? sc.y : 8);
  *z_values = N >= 2048 ? 8 : (sc.z ? sc.z : 8);
  return PK_OK;
}

// Average duration in ms of `reps` launches of one pass with column schedule `e`.
static pk_status time_pass(Plan p, int which, int e, char* ws, int reps, hipStream_t s, hipEvent_t a, hipEvent_t b,
                           float* ms) {
  p.col_e[which] = e;
  // the y pass is timed on the last slab, whose x-transformed rows X still holds
  const int z0 = p.N - p.xs, pb = ((p.N / p.xs - 1) % p.xr) * p.xs;
  hipError_t err = which == 0 ? launch_ypass(p, ws, s, z0, pb) : launch_zpass(p, ws, s);  // warm-up
  if (err != hipSuccess) return hip_fail(err, "autotune warm-up");
  if ((err = hipEventRecord(a, s)) != hipSuccess) return hip_fail(err, "event record");
  for (int r = 0; r < reps; ++r) {
    err = which == 0 ? launch_ypass(p, ws, s, z0, pb) : launch_zpass(p, ws, s);
    if (err != hipSuccess) return hip_fail(err, "autotune launch");
  }
  if ((err = hipEventRecord(b, s)) != hipSuccess) return hip_fail(err, "event record");
  if ((err = hipEventSynchronize(b)) != hipSuccess) return hip_fail(err, "event synchronize");
  if ((err = hipEventElapsedTime(ms, a, b)) != hipSuccess) return hip_fail(err, "event time");
  *ms /= (float)reps;
  return PK_OK;
}

pk_status pk_autotune(const pk_config* cfg, const pk_catalog* gal, const pk_catalog* ran, void* workspace,
                      size_t workspace_bytes, int32_t reps, int32_t* y_values, int32_t* z_values, void* hip_stream) {
  if (reps < 1) return fail(PK_EINVAL, "reps must be >= 1");
  if (!y_values || !z_values) return fail(PK_EINVAL, "null output pointer");
  pk_result dummy;
  memset(&dummy, 0, sizeof(dummy));
  // one full run validates the inputs and leaves the grids the passes read in the workspace
  pk_status st = pk_multipoles(cfg, gal, ran, workspace, workspace_bytes, &dummy, hip_stream);
  if (st != PK_OK) return st;
  Plan p;
  st = prepare(cfg, gal, ran, workspace, workspace_bytes, &p);
  if (st != PK_OK) return st;
  hipStream_t s = (hipStream_t)hip_stream;
  hipEvent_t a = nullptr, b = nullptr;
  hipError_t err;
  if ((err = hipEventCreate(&a)) != hipSuccess) return hip_fail(err, "event create");
  if ((err = hipEventCreate(&b)) != hipSuccess) {
    hipEventDestroy(a);
    return hip_fail(err, "event create");
  }
  const int cand[2] = {16, 8};
  const int k0 = p.N >= 2048 ? 1 : 0;  // 8 only at 2048
  int best[2] = {cand[k0], cand[k0]};
  for (int which = 0; which < 2 && st == PK_OK; ++which) {
    float tbest = 0.0f;
    for (int k = k0; k < 2 && st == PK_OK; ++k) {
      float ms = 0.0f;
      st = time_pass(p, which, cand[k], static_cast<char*>(workspace), reps, s, a, b, &ms);
      if (st == PK_OK && (k == k0 || ms < tbest)) {
        tbest = ms;
        best[which] = cand[k];
      }
    }
  }
  hipEventDestroy(a);
  hipEventDestroy(b);
  if (st != PK_OK) return st;
  g_sched[log2_of(p.N)][p.ell_max / 2] = Schedule{best[0], best[1]};
  *y_values = best[0];
  *z_values = best[1];
  return PK_OK;
}

// ------------------------------------------------------------------------- batches

static pk_status batch_layout(const pk_config* cfgs, const pk_catalog* gals, const pk_catalog* rans, int32_t n,
                              int32_t lanes, size_t* lane_bytes, int64_t* rd_max, size_t* total) {
  if (!cfgs || !gals || !rans) return fail(PK_EINVAL, "null batch array");
  if (n < 0) return fail(PK_EINVAL, "n_mocks < 0");
  if (lanes < 1 || lanes > 2) return fail(PK_EINVAL, "lanes must be 1 or 2");
  size_t wmax = 256;
  int64_t rmax = 1;
  for (int32_t i = 0; i < n; ++i) {
    Plan p;
    const char* why;
    pk_status st = check_catalog(&gals[i], cfgs[i].norm_from == 1, "galaxy");
    if (st == PK_OK) st = check_catalog(&rans[i], cfgs[i].norm_from == 0, "random");
    if (st == PK_OK) st = make_plan(&cfgs[i], gals[i].n, rans[i].n, &p, &why);
    if (st != PK_OK) return fail(st, "mock " + std::to_string(i) + ": " + g_last_error);
    if (p.total > wmax) wmax = p.total;
    if (p.result_doubles > rmax) rmax = p.result_doubles;
  }
  *lane_bytes = align256(wmax);
  *rd_max = rmax;
  *total = (size_t)lanes * *lane_bytes + align256(sizeof(double) * (size_t)rmax * (n > 0 ? n : 1));
  return PK_OK;
}

struct GraphSlot {
  bool valid = false;
  int key[9] = {0};
  hipGraphExec_t exec = nullptr;
};

static void class_key(const Plan& p, int (&k)[9]) {
  k[0] = p.N; k[1] = p.assign; k[2] = p.ell_max; k[3] = p.nbins; k[4] = p.dn; k[5] = p.los; k[6] = p.compensate;
  k[7] = p.norm_from; k[8] = p.xs;
}

}  // extern "C"

static pk_status batch_fail_cleanup(pk_status st, hipStream_t* ls, int lanes, GraphSlot* gs, hipEvent_t* ev, int nev) {
  for (int l = 0; l < lanes; ++l) {
    if (gs[l].exec) hipGraphExecDestroy(gs[l].exec);
    if (ls[l]) hipStreamDestroy(ls[l]);
  }
  for (int i = 0; i < nev; ++i)
    if (ev[i]) hipEventDestroy(ev[i]);
  return st;
}

extern "C" {

pk_status pk_workspace_size_batch(const pk_config* cfgs, const pk_catalog* gals, const pk_catalog* rans,
                                  int32_t n_mocks, int32_t lanes, size_t* bytes) {
  if (!bytes) return fail(PK_EINVAL, "null bytes pointer");
  size_t lane_bytes, total;
  int64_t rd;
  const pk_status st = batch_layout(cfgs, gals, rans, n_mocks, lanes, &lane_bytes, &rd, &total);
  if (st == PK_OK) *bytes = total;
  return st;
}

pk_status pk_multipoles_batch(const pk_config* cfgs, const pk_catalog* gals, const pk_catalog* rans, int32_t n_mocks,
                              int32_t lanes, void* workspace, size_t workspace_bytes, pk_result* outs,
                              pk_status* per_mock, void* hip_stream) {
  size_t lane_bytes, total;
  int64_t rd;
  pk_status st = batch_layout(cfgs, gals, rans, n_mocks, lanes, &lane_bytes, &rd, &total);
  if (st != PK_OK) return st;
  if (!outs || !per_mock) return fail(PK_EINVAL, "null outs or per_mock");
  if (!workspace || workspace_bytes < total)
    return fail(PK_EWORKSPACE, "batch workspace needs " + std::to_string(total) + " bytes");
  if (((uintptr_t)workspace & 255) != 0) return fail(PK_EWORKSPACE, "workspace must be 256-byte aligned");
  if (n_mocks == 0) return PK_OK;
  char* ws = static_cast<char*>(workspace);
  double* d_res = at<double>(ws, (size_t)lanes * lane_bytes);
  hipStream_t caller = (hipStream_t)hip_stream;
  hipStream_t ls[2] = {nullptr, nullptr};
  GraphSlot gs[2];
  hipEvent_t ev[3] = {nullptr, nullptr, nullptr};
  hipError_t e;
  for (int i = 0; i < 3; ++i)
    if ((e = hipEventCreateWithFlags(&ev[i], hipEventDisableTiming)) != hipSuccess)
      return batch_fail_cleanup(hip_fail(e, "event create"), ls, lanes, gs, ev, 3);
  for (int l = 0; l < lanes; ++l)
    if ((e = hipStreamCreateWithFlags(&ls[l], hipStreamNonBlocking)) != hipSuccess)
      return batch_fail_cleanup(hip_fail(e, "stream create"), ls, lanes, gs, ev, 3);
  // lanes start after the caller's queued work
  if ((e = hipEventRecord(ev[0], caller)) != hipSuccess) return batch_fail_cleanup(hip_fail(e, "record"), ls, lanes, gs, ev, 3);
  for (int l = 0; l < lanes; ++l) hipStreamWaitEvent(ls[l], ev[0], 0);
  const bool timing = g_timing.enabled;
  g_timing.enabled = false;  // no per-stage events inside captured graphs
  for (int32_t i = 0; i < n_mocks; ++i) {
    const int l = i % lanes;
    Plan p;
    const char* why;
    make_plan(&cfgs[i], gals[i].n, rans[i].n, &p, &why);
    char* lws = ws + (size_t)l * lane_bytes;
    hipGraph_t graph = nullptr;
    if ((e = hipStreamBeginCapture(ls[l], hipStreamCaptureModeThreadLocal)) != hipSuccess) {
      g_timing.enabled = timing;
      return batch_fail_cleanup(hip_fail(e, "begin capture"), ls, lanes, gs, ev, 3);
    }
    st = run_stages(p, gals[i], rans[i], lws, d_res + (size_t)i * rd, ls[l], Stop::kNone);
    e = hipStreamEndCapture(ls[l], &graph);
    if (st != PK_OK || e != hipSuccess) {
      if (graph) hipGraphDestroy(graph);
      g_timing.enabled = timing;
      return batch_fail_cleanup(st != PK_OK ? st : hip_fail(e, "end capture"), ls, lanes, gs, ev, 3);
    }
    int key[9];
    class_key(p, key);
    bool reused = false;
    if (gs[l].valid && memcmp(gs[l].key, key, sizeof(key)) == 0) {
      hipGraphExecUpdateResult res;
      hipGraphNode_t bad = nullptr;
      reused = hipGraphExecUpdate(gs[l].exec, graph, &bad, &res) == hipSuccess && res == hipGraphExecUpdateSuccess;
    }
    if (!reused) {
      if (gs[l].exec) hipGraphExecDestroy(gs[l].exec);
      gs[l].exec = nullptr;
      gs[l].valid = false;
      if ((e = hipGraphInstantiate(&gs[l].exec, graph, nullptr, nullptr, 0)) != hipSuccess) {
        hipGraphDestroy(graph);
        g_timing.enabled = timing;
        return batch_fail_cleanup(hip_fail(e, "graph instantiate"), ls, lanes, gs, ev, 3);
      }
      memcpy(gs[l].key, key, sizeof(key));
      gs[l].valid = true;
    }
    hipGraphDestroy(graph);
    if ((e = hipGraphLaunch(gs[l].exec, ls[l])) != hipSuccess) {
      g_timing.enabled = timing;
      return batch_fail_cleanup(hip_fail(e, "graph launch"), ls, lanes, gs, ev, 3);
    }
  }
  g_timing.enabled = timing;
  // the caller's stream waits for every lane
  for (int l = 0; l < lanes; ++l) {
    hipEventRecord(ev[1 + l], ls[l]);
    hipStreamWaitEvent(caller, ev[1 + l], 0);
  }
  std::vector<double> h((size_t)rd * n_mocks);
  e = hipMemcpyAsync(h.data(), d_res, sizeof(double) * h.size(), hipMemcpyDeviceToHost, caller);
  if (e == hipSuccess) e = hipStreamSynchronize(caller);
  if (e != hipSuccess) return batch_fail_cleanup(hip_fail(e, "batch results"), ls, lanes, gs, ev, 3);
  batch_fail_cleanup(PK_OK, ls, lanes, gs, ev, 3);
  for (int32_t i = 0; i < n_mocks; ++i) {
    const double* r = h.data() + (size_t)i * rd;
    per_mock[i] = unpack_result(r, cfgs[i].nbins, cfgs[i].ell_max / 2 + 1, &outs[i]);
  }
  return PK_OK;
}

pk_status pk_stage_xgrids(const pk_config* cfg, const pk_catalog* gal, const pk_catalog* ran, void* workspace,
                          size_t workspace_bytes, void* hip_stream) {
  Plan p;
  pk_status st = prepare(cfg, gal, ran, workspace, workspace_bytes, &p);
  if (st != PK_OK) return st;
  return run_stages(p, *gal, *ran, static_cast<char*>(workspace), nullptr, (hipStream_t)hip_stream, Stop::kAfterX);
}

pk_status pk_stage_fft(const pk_config* cfg, const pk_catalog* gal, const pk_catalog* ran, void* workspace,
                       size_t workspace_bytes, void* hip_stream) {
  Plan p;
  pk_status st = prepare(cfg, gal, ran, workspace, workspace_bytes, &p);
  if (st != PK_OK) return st;
  return run_stages(p, *gal, *ran, static_cast<char*>(workspace), nullptr, (hipStream_t)hip_stream, Stop::kAfterY);
}

pk_status pk_stage_contract(const pk_config* cfg, int64_t n_gal, int64_t n_ran, void* workspace,
                            size_t workspace_bytes, pk_result* out, void* hip_stream) {
  Plan p;
  const char* why;
  pk_status st = make_plan(cfg, n_gal, n_ran, &p, &why);
  if (st != PK_OK) return st;
  if (!out) return fail(PK_EINVAL, "null result");
  if (!workspace || workspace_bytes < p.total)
    return fail(PK_EWORKSPACE, "workspace needs " + std::to_string(p.total) + " bytes, got " +
                                   std::to_string(workspace_bytes));
  if (((uintptr_t)workspace & 255) != 0) return fail(PK_EWORKSPACE, "workspace must be 256-byte aligned");
  char* ws = static_cast<char*>(workspace);
  hipStream_t s = (hipStream_t)hip_stream;
  double* d_res = at<double>(ws, p.off_result);
  hipError_t e;
  if ((e = launch_zpass(p, ws, s)) != hipSuccess) return hip_fail(e, "z transform and binning");
  if ((e = launch_finalize(p, ws, d_res, s)) != hipSuccess) return hip_fail(e, "finalize");
  return fetch_result(p, d_res, s, out);
}

pk_status pk_hgrid_layout(const pk_config* cfg, int64_t n_gal, int64_t n_ran, int32_t group, int32_t kx_tile,
                          size_t* offset, int32_t* ky_max, int32_t* tile_cols) {
  Plan p;
  const char* why;
  pk_status st = make_plan(cfg, n_gal, n_ran, &p, &why);
  if (st != PK_OK) return st;
  if (group < 0 || group >= p.groups.ngroups) return fail(PK_EINVAL, "group index out of range");
  if (kx_tile < 0 || kx_tile >= p.nkt) return fail(PK_EINVAL, "kx tile out of range");
  if (!offset || !ky_max || !tile_cols) return fail(PK_EINVAL, "null output pointer");
  *offset = p.off_H + sizeof(float) * 2 * ((size_t)group * p.H_group_stride + (size_t)p.tiles.regoff[kx_tile]);
  *ky_max = p.tiles.M[kx_tile];
  *tile_cols = p.TK;
  return PK_OK;
}

int32_t pk_ygroup_terms(int32_t ell_max, int32_t max_groups, int32_t cap, int32_t* set, int32_t* group,
                        int32_t* grid, float* coef, int32_t* a, int32_t* b) {
  if (!ell_ok(ell_max) || (max_groups != 3 && max_groups != kYSetGroups) || cap < 0 ||
      (cap > 0 && (!set || !group || !grid || !coef || !a || !b))) {
    fail(PK_EINVAL, "bad ell_max, max_groups or output arrays");
    return -1;
  }
  GroupTable gt;
  YSetTable yt;
  build_groups(ell_max, &gt);
  build_ysets(gt, ell_max, max_groups, &yt);
  int32_t k = 0;
  for (int s = 0; s < yt.nsets; ++s)
    for (int i = yt.mem0[s]; i < yt.mem0[s + 1]; ++i)
      for (int q = yt.term0[i]; q < yt.term0[i + 1]; ++q, ++k)
        if (k < cap) {
          set[k] = s;
          group[k] = yt.group[s][yt.tslot[q]];
          grid[k] = kept_monomial(yt.mgrid[i]);
          coef[k] = yt.tcoef[q];
          a[k] = yt.ta[q];
          b[k] = yt.tb[q];
        }
  return k;
}

pk_status pk_zgroup(int32_t ell_max, int32_t group, int32_t* degree, int32_t* z_power) {
  if (!ell_ok(ell_max) || !degree || !z_power) return fail(PK_EINVAL, "bad ell_max or null pointer");
  int g = 0;
  for (int n = 0; n <= ell_max; n += 2)
    for (int c = 0; c <= n; ++c, ++g)
      if (g == group) {
        *degree = n;
        *z_power = c;
        return PK_OK;
      }
  return fail(PK_EINVAL, "group index out of range");
}

pk_status pk_xgrid_layout(const pk_config* cfg, int64_t n_gal, int64_t n_ran, int32_t m, size_t* offset,
                          int32_t* kx_count) {
  Plan p;
  const char* why;
  pk_status st = make_plan(cfg, n_gal, n_ran, &p, &why);
  if (st != PK_OK) return st;
  if (m < 0 || m >= p.G) return fail(PK_EINVAL, "grid index out of range");
  if (!offset || !kx_count) return fail(PK_EINVAL, "null output pointer");
  int j = -1;
  for (int i = 0; i < p.GK; ++i)
    if (kept_monomial(i) == m) j = i;
  if (j < 0) return fail(PK_EINVAL, "grid not stored: its power of rhat_z is 2 or more (it follows from the stored ones)");
  *offset = p.off_X + sizeof(float) * 2 * (size_t)j * p.xr * p.xs * p.N * p.Kx;
  *kx_count = p.Kx;
  return PK_OK;
}

pk_status pk_x_planes(const pk_config* cfg, int64_t n_gal, int64_t n_ran, int32_t* planes) {
  if (!planes) return fail(PK_EINVAL, "null output pointer");
  Plan p;
  const char* why;
  pk_status st = make_plan(cfg, n_gal, n_ran, &p, &why);
  if (st != PK_OK) return st;
  *planes = p.xs;
  return PK_OK;
}

pk_status pk_set_stage_timing(int32_t enable) {
  g_timing.enabled = enable != 0;
  return PK_OK;
}

int32_t pk_stage_times(double* ms, int32_t n) {
  if (!g_timing.recorded) return -1;
  if (hipEventSynchronize(g_timing.ev[kNumStages]) != hipSuccess) return -1;
  for (int i = 0; i < kNumStages && i < n; ++i) {
    float t = 0.0f;
    if (hipEventElapsedTime(&t, g_timing.ev[i], g_timing.ev[i + 1]) != hipSuccess) return -1;
    if (ms) ms[i] = t;
  }
  return kNumStages;
}

const char* pk_stage_name(int32_t i) { return (i >= 0 && i < kNumStages) ? kStageNames[i] : "?"; }

int32_t pk_num_grids(int32_t ell_max) {
  return ell_ok(ell_max) ? num_grids_for(ell_max) : -1;
}

pk_status pk_monomial(int32_t m, int32_t* a, int32_t* b, int32_t* c) {
  if (m < 0 || m >= kMaxGrids || !a || !b || !c) return fail(PK_EINVAL, "bad monomial index or null pointer");
  const Monomial mo = monomial(m);
  *a = mo.a;
  *b = mo.b;
  *c = mo.c;
  return PK_OK;
}

const char* pk_status_string(pk_status s) {
  switch (s) {
    case PK_OK: return "ok";
    case PK_EINVAL: return "invalid argument";
    case PK_ERANGE: return "particle outside the box";
    case PK_EDOM: return "invalid input value";
    case PK_EWORKSPACE: return "workspace too small";
    case PK_EDEVICE: return "HIP runtime error";
    case PK_ENOTSUP: return "unsupported size";
    default: return "unknown status";
  }
}

size_t pk_last_error(char* buf, size_t n) {
  if (buf && n > 0) {
    const size_t k = g_last_error.size() < n - 1 ? g_last_error.size() : n - 1;
    memcpy(buf, g_last_error.data(), k);
    buf[k] = '\0';
  }
  return g_last_error.size();
}

size_t pk_last_error_detail(char* buf, size_t n) { return pk_last_error(buf, n); }

}  // extern "C"
