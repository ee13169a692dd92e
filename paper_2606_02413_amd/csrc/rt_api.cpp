// C ABI: argument and value validation on the host, model staging, and the
// launch plan of a trace call.  All device work is ordered on the caller's
// stream.
#include <hip/hip_runtime.h>

#include <atomic>
#include <cmath>
#include <algorithm>
#include <cstdlib>
#include <cstring>
#include <memory>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "rt_internal.hpp"
#include "rt_probe.hpp"

using namespace rt;

namespace {

thread_local std::string g_err;

rt_status fail(rt_status s, const std::string& msg) {
  g_err = msg;
  return s;
}

std::atomic<long long> g_device_bytes{0};

long long env_bytes(const char* name) {
  const char* e = std::getenv(name);
  if (!e || !*e) return -1;
  char* end = nullptr;
  long long v = std::strtoll(e, &end, 10);
  return (end && *end == '\0' && v >= 0) ? v : -1;
}

long long byte_cap() { return env_bytes("RT_MAX_DEVICE_BYTES"); }

// Allocation through one place so the optional byte cap applies everywhere.
rt_status dev_alloc(void** p, size_t bytes, const char* what) {
  const long long cap = byte_cap();
  if (cap >= 0 && g_device_bytes.load() + (long long)bytes > cap)
    return fail(RT_E_OUT_OF_MEMORY, std::string(what) + ": RT_MAX_DEVICE_BYTES exceeded");
  hipError_t e = hipMalloc(p, bytes);
  if (e == hipErrorOutOfMemory) return fail(RT_E_OUT_OF_MEMORY, std::string(what) + ": hipMalloc out of memory");
  if (e != hipSuccess) return fail(RT_E_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
  g_device_bytes += (long long)bytes;
  return RT_OK;
}

void dev_free(void* p, size_t bytes) {
  if (!p) return;
  (void)hipFree(p);
  g_device_bytes -= (long long)bytes;
}

rt_status hip_check(hipError_t e, const char* what) {
  if (e == hipSuccess) return RT_OK;
  return fail(RT_E_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

bool finite3(const double* v) { return std::isfinite(v[0]) && std::isfinite(v[1]) && std::isfinite(v[2]); }

// Library-owned device tables of the trace calls.
//
// A block that a call outgrows is retired, not freed: a HIP graph captured
// earlier may still launch kernels that read it, so retired blocks stay
// allocated until the process ends.  Every call rewrites the contents it reads
// (launch table, start n_e, counters) before reading them, on its own stream.
struct Block {
  void* p = nullptr;
  size_t bytes = 0;
};

// The tables of one stream.  Calls on one stream run in order and share them;
// calls on different streams use different tables, so they do not race.
struct StreamTables {
  hipStream_t stream = nullptr;
  unsigned* counters = nullptr;  // kXcds claim counters (persistent trace, adjoint sweep)
  Block launch;                  // per-pixel start point and grid index, 48 B a pixel
  Block start_ne;                // n_e at the start point per (model, pixel)
  Block path_rays;               // device copy of a call's path-ray list
  Block blur_tmp;                // intermediate maps of the beam convolution
  Block adj;                     // adjoint workspace (freed when outgrown: the adjoint refuses capture)
};

struct DeviceScratch {
  int n_cu = 0;
  rt_tuning tune{RT_ABI_VERSION, 64, 0, kXcds};  // launch tuning of the persistent trace
  std::vector<std::unique_ptr<StreamTables>> streams;
  std::vector<Block> retired;
};
constexpr long long kAdjMaxCheckpoints = 128;  // per ray; longer rays thin their checkpoints
constexpr long long kAdjCheckpointBudget = 8ll << 30;  // bytes of per-ray checkpoints per batch of tiles
std::mutex g_scratch_mu;
DeviceScratch g_scratch[64];

// Fixed device scratch of rt_trace_maps_static: one array per device, held from
// the library's load on that device until the process ends.  Host code never
// uses the array's name as an address: the device address comes from
// hipGetSymbolAddress, once per device (g_static_ptr).
constexpr size_t kStaticScratchBytes = size_t(RT_STATIC_SCRATCH_BYTES);
constexpr size_t kStaticCountersBytes = 256;  // kXcds claim counters, padded
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];
void* g_static_ptr[64] = {};


// Call with g_scratch_mu held.
rt_status scratch_for(int dev, DeviceScratch** out) {
  if (dev < 0 || dev >= 64) return fail(RT_E_DEVICE, "device index out of range");
  DeviceScratch& s = g_scratch[dev];
  if (s.n_cu == 0) {
    int n = 0;
    if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n < 1) n = 1;
    s.n_cu = n;
  }
  *out = &s;
  return RT_OK;
}

// Call with g_scratch_mu held and `dev` current.
rt_status tables_for(int dev, hipStream_t stream, DeviceScratch** sc_out, StreamTables** out) {
  DeviceScratch* sc = nullptr;
  rt_status st = scratch_for(dev, &sc);
  if (st != RT_OK) return st;
  *sc_out = sc;
  for (auto& t : sc->streams)
    if (t->stream == stream) {
      *out = t.get();
      return RT_OK;
    }
  std::unique_ptr<StreamTables> t(new (std::nothrow) StreamTables());
  if (!t) return fail(RT_E_OUT_OF_MEMORY, "host allocation");
  t->stream = stream;
  void* p = nullptr;
  st = dev_alloc(&p, sizeof(unsigned) * kXcds, "work-queue counters");
  if (st != RT_OK) return st;
  t->counters = static_cast<unsigned*>(p);
  *out = t.get();
  sc->streams.push_back(std::move(t));
  return RT_OK;
}

// Grow a block to at least `need` bytes; the outgrown block is retired (kept
// allocated) unless `can_free`.  Call with g_scratch_mu held.
rt_status grow(DeviceScratch* sc, Block& b, size_t need, const char* what, bool can_free = false) {
  if (b.bytes >= need) return RT_OK;
  if (b.p) {
    if (can_free) dev_free(b.p, b.bytes);
    else sc->retired.push_back(b);
  }
  b = Block{};
  void* p = nullptr;
  rt_status st = dev_alloc(&p, need, what);
  if (st != RT_OK) return st;
  b.p = p;
  b.bytes = need;
  return RT_OK;
}

}  // namespace

struct rt_model {
  rt_grid_desc desc;
  DevGeom geom;
  int device;
  float4* nfg;
  float* te;
  size_t nfg_bytes, te_bytes;
  float* raw_ne;  // staging copies of the input arrays (C-order)
  float* raw_te;
  size_t raw_bytes;
  int* bad;       // invalid-value counter of device-side updates
};

namespace {

rt_status validate_desc(const rt_grid_desc* d) {
  if (!d) return fail(RT_E_INVALID_ARG, "desc is NULL");
  if (d->abi_version != RT_ABI_VERSION) return fail(RT_E_INVALID_ARG, "desc->abi_version mismatch");
  if (d->kind == RT_GRID_SPHERICAL_LOGR) {
    if (d->n0 < 2 || d->n1 < 2 || d->n2 < 3) return fail(RT_E_INVALID_ARG, "spherical grid needs n0, n1 >= 2, n2 >= 3");
    if (!(std::isfinite(d->r_in) && std::isfinite(d->r_max) && d->r_in > 0.0 && d->r_max > d->r_in))
      return fail(RT_E_INVALID_ARG, "spherical grid needs 0 < r_in < r_max");
  } else if (d->kind == RT_GRID_CARTESIAN) {
    if (d->n0 < 2 || d->n1 < 2 || d->n2 < 2) return fail(RT_E_INVALID_ARG, "Cartesian grid needs n >= 2 per axis");
    if (!finite3(d->origin) || !finite3(d->spacing)) return fail(RT_E_INVALID_ARG, "origin/spacing not finite");
    for (int k = 0; k < 3; ++k)
      if (!(d->spacing[k] > 0.0)) return fail(RT_E_INVALID_ARG, "spacing must be > 0");
    if (!(std::isfinite(d->r_in) && std::isfinite(d->r_max) && d->r_max > 0.0 && d->r_in < d->r_max))
      return fail(RT_E_INVALID_ARG, "need r_in < r_max, r_max > 0");
  } else {
    return fail(RT_E_INVALID_ARG, "unknown grid kind");
  }
  // The kernels form a cell's key (a n1 + b) n2p + c with 24-bit multiplies and
  // keep keys in 32-bit ints: n0 n1 and the packed row length n2p (n2 + 1 on
  // spherical grids) must stay below 2^24, and n0 n1 n2p below 2^31.
  const long long n2p = d->kind == RT_GRID_SPHERICAL_LOGR ? (long long)d->n2 + 1 : (long long)d->n2;
  if ((long long)d->n0 * d->n1 >= (1ll << 24) || n2p >= (1ll << 24))
    return fail(RT_E_CAPACITY, "grid needs n0*n1 < 2^24 and a packed row length below 2^24");
  if ((long long)d->n0 * d->n1 * n2p > (1ll << 31) - 1)
    return fail(RT_E_CAPACITY, "grid has more than 2^31-1 packed vertices");
  return RT_OK;
}

rt_status validate_values_host(const float* ne, const float* te, long long n) {
  for (long long i = 0; i < n; ++i) {
    const float x = ne[i], t = te[i];
    if (!(std::isfinite(x) && x >= 0.0f)) return fail(RT_E_NONFINITE_INPUT, "n_e[" + std::to_string(i) + "] is not finite and >= 0");
    if (!(std::isfinite(t) && t > 0.0f)) return fail(RT_E_NONFINITE_INPUT, "T[" + std::to_string(i) + "] is not finite and > 0");
  }
  return RT_OK;
}

DevGeom make_geom(const rt_grid_desc& d) {
  DevGeom g{};
  g.kind = int(d.kind);
  g.n0 = d.n0; g.n1 = d.n1; g.n2 = d.n2;
  g.n2p = (d.kind == RT_GRID_SPHERICAL_LOGR) ? d.n2 + 1 : d.n2;
  if (d.kind == RT_GRID_SPHERICAL_LOGR) {
    const double dl = std::log(d.r_max / d.r_in) / double(d.n0 - 1);
    g.ln_rin_d = std::log(d.r_in);
    g.inv_dl_d = 1.0 / dl;
    g.inv_dth_d = double(d.n1) / M_PI;
    g.inv_dph_d = double(d.n2) / (2.0 * M_PI);
    g.ln_rin = float(g.ln_rin_d);
    g.inv_dl = float(g.inv_dl_d);
    g.inv_dth = float(g.inv_dth_d);
    g.inv_dph = float(g.inv_dph_d);
    g.has_inner = 1;
  } else {
    for (int k = 0; k < 3; ++k) {
      g.org_d[k] = d.origin[k];
      g.inv_sp_d[k] = 1.0 / d.spacing[k];
      g.org[k] = float(g.org_d[k]);
      g.inv_sp[k] = float(g.inv_sp_d[k]);
    }
    g.has_inner = d.r_in > 0.0 ? 1 : 0;
  }
  g.r_in = d.r_in;
  g.r_max = d.r_max;
  return g;
}

bool same_grid(const rt_grid_desc& a, const rt_grid_desc& b) {
  if (a.kind != b.kind || a.n0 != b.n0 || a.n1 != b.n1 || a.n2 != b.n2 || a.r_in != b.r_in || a.r_max != b.r_max)
    return false;
  if (a.kind == RT_GRID_CARTESIAN)
    for (int k = 0; k < 3; ++k)
      if (a.origin[k] != b.origin[k] || a.spacing[k] != b.spacing[k]) return false;
  return true;
}

rt_status stage_model(rt_model* m, hipStream_t s) {
  hipError_t e = launch_pack(m->geom, m->raw_ne, m->raw_te, m->nfg, m->te, s);
  if (e != hipSuccess) return hip_check(e, "pack kernel");
  return hip_check(hipStreamSynchronize(s), "model staging");
}

void free_model_memory(rt_model* m) {
  dev_free(m->nfg, m->nfg_bytes);
  dev_free(m->te, m->te_bytes);
  dev_free(m->raw_ne, m->raw_bytes);
  dev_free(m->raw_te, m->raw_bytes);
  dev_free(m->bad, sizeof(int));
  m->nfg = nullptr; m->te = nullptr; m->raw_ne = nullptr; m->raw_te = nullptr; m->bad = nullptr;
}


// Validation of a trace call (host only) and the parts of its launch plan that
// the forward and the adjoint share: geometry, frequencies, image axes, stepping
// controls and the per-pixel launch table.
rt_status validate_call(const rt_model* const* models, int32_t n_models, const double* freq_hz, int32_t n_freq,
                        const rt_image_desc* image, const rt_params* params, TraceArgs& a) {
  if (!models || n_models < 1) return fail(RT_E_INVALID_ARG, "need at least one model");
  if (!freq_hz || n_freq < 1) return fail(RT_E_INVALID_ARG, "need at least one frequency");
  if (!image || !params) return fail(RT_E_INVALID_ARG, "image/params is NULL");
  for (int k = 0; k < n_models; ++k)
    if (!models[k]) return fail(RT_E_INVALID_ARG, "models[" + std::to_string(k) + "] is NULL");
  const rt_model* m0 = models[0];
  for (int k = 1; k < n_models; ++k) {
    if (!same_grid(models[k]->desc, m0->desc)) return fail(RT_E_INVALID_ARG, "models must share one grid descriptor");
    if (models[k]->device != m0->device) return fail(RT_E_INVALID_ARG, "models must be on one device");
  }
  for (int k = 0; k < n_freq; ++k)
    if (!(std::isfinite(freq_hz[k]) && freq_hz[k] > 0.0)) return fail(RT_E_INVALID_ARG, "frequencies must be finite and > 0");
  if (n_models > kMaxModels) return fail(RT_E_CAPACITY, "more than 16 models in one call");
  if (n_freq > kMaxFreqs) return fail(RT_E_CAPACITY, "more than 128 frequencies in one call");
  const rt_params& P = *params;
  if (P.abi_version != RT_ABI_VERSION) return fail(RT_E_INVALID_ARG, "params->abi_version mismatch");
  const uint32_t known = RT_USE_MAGNIFICATION | RT_USE_REFRACTION | RT_PREC_ALL_FP32 | RT_PREC_FP32_STEP |
                         RT_SCHED_PLAIN | RT_DETERMINISTIC_GRAD | RT_CARRIED_TUBE | RT_TEST_NO_ABSORPTION;
  if (P.flags & ~known) return fail(RT_E_INVALID_ARG, "unknown flag bits");
  if (P.flags & RT_CARRIED_TUBE) {
    if ((P.flags & (RT_USE_REFRACTION | RT_USE_MAGNIFICATION)) != (RT_USE_REFRACTION | RT_USE_MAGNIFICATION))
      return fail(RT_E_INVALID_ARG, "RT_CARRIED_TUBE needs RT_USE_REFRACTION and RT_USE_MAGNIFICATION");
    if (P.flags & (RT_PREC_ALL_FP32 | RT_PREC_FP32_STEP))
      return fail(RT_E_UNSUPPORTED, "RT_CARRIED_TUBE runs in the default precision only");
  }
  if (!(std::isfinite(P.ds_max) && P.ds_max > 0.0)) return fail(RT_E_INVALID_ARG, "ds_max must be > 0");
  if (!(std::isfinite(P.n_floor) && P.n_floor > 0.0 && P.n_floor <= 1.0)) return fail(RT_E_INVALID_ARG, "n_floor must be in (0, 1]");
  if (P.max_steps < 1) return fail(RT_E_INVALID_ARG, "max_steps must be >= 1");
  if (!(std::isfinite(P.perturb_ratio) && P.perturb_ratio > 0.0)) return fail(RT_E_INVALID_ARG, "perturb_ratio must be > 0");
  if (!(std::isfinite(P.tb_inner_K) && std::isfinite(P.tb_sky_K))) return fail(RT_E_INVALID_ARG, "boundary temperatures must be finite");
  const rt_image_desc& I = *image;
  if (I.nu < 1 || I.nv < 1) return fail(RT_E_INVALID_ARG, "image needs nu, nv >= 1");
  if (!(std::isfinite(I.half_u) && std::isfinite(I.half_v) && I.half_u > 0 && I.half_v > 0))
    return fail(RT_E_INVALID_ARG, "image half widths must be > 0");
  if (!finite3(I.obs_dir) || !finite3(I.up)) return fail(RT_E_INVALID_ARG, "obs_dir/up not finite");
  double o[3] = {I.obs_dir[0], I.obs_dir[1], I.obs_dir[2]};
  const double on = std::sqrt(o[0] * o[0] + o[1] * o[1] + o[2] * o[2]);
  if (!(on > 0)) return fail(RT_E_INVALID_ARG, "obs_dir is zero");
  for (double& x : o) x /= on;
  double u[3] = {I.up[1] * o[2] - I.up[2] * o[1], I.up[2] * o[0] - I.up[0] * o[2], I.up[0] * o[1] - I.up[1] * o[0]};
  const double un = std::sqrt(u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
  if (!(un > 1e-12)) return fail(RT_E_INVALID_ARG, "up is parallel to obs_dir");
  for (double& x : u) x /= un;
  const double v[3] = {o[1] * u[2] - o[2] * u[1], o[2] * u[0] - o[0] * u[2], o[0] * u[1] - o[1] * u[0]};
  const long long npx = (long long)I.nu * I.nv;
  const long long total = npx * n_models * n_freq;
  if (total > (1ll << 31) - 1) return fail(RT_E_CAPACITY, "more than 2^31-1 rays in one call");

  a.g = m0->geom;
  for (int k = 0; k < n_models; ++k) a.models[k] = {models[k]->nfg, models[k]->te};
  for (int k = 0; k < n_freq; ++k) {
    a.freqs[k] = freq_hz[k];
    a.xf[k] = (8.98e3 / freq_hz[k]) * (8.98e3 / freq_hz[k]);
    a.lnf[k] = float(std::log(freq_hz[k]));
  }
  a.n_models = n_models;
  a.n_freq = n_freq;
  a.nu = I.nu; a.nv = I.nv;
  a.tiles_u = (I.nu + kTile - 1) / kTile;
  a.tiles_v = (I.nv + kTile - 1) / kTile;
  a.tiles_per_image = a.tiles_u * a.tiles_v;
  for (int k = 0; k < 3; ++k) { a.o[k] = o[k]; a.u[k] = u[k]; a.v[k] = v[k]; }
  a.half_u = I.half_u; a.half_v = I.half_v;
  a.ds_max = float(P.ds_max);
  a.n_floor = float(P.n_floor);
  a.ds_max_d = P.ds_max;
  a.n_floor_d = P.n_floor;
  a.eta = float(P.perturb_ratio);
  a.max_steps = P.max_steps;
  a.tb_inner = P.tb_inner_K;
  a.tb_sky = P.tb_sky_K;
  a.flags = P.flags;
  return RT_OK;
}

// Bytes of the per-call tables a validated call reads: launch table and start n_e.
size_t launch_table_bytes(const TraceArgs& a) { return size_t(a.nu) * size_t(a.nv) * 6 * sizeof(double); }
size_t start_ne_bytes(const TraceArgs& a) { return size_t(a.nu) * size_t(a.nv) * size_t(a.n_models) * sizeof(float); }

// The stream's tables for a validated call, grown to its size, and the launch
// table and start n_e written on the stream.
rt_status prepare_call(const rt_model* const* models, int32_t n_models, const double* freq_hz, int32_t n_freq,
                       const rt_image_desc* image, const rt_params* params, hipStream_t s, TraceArgs& a,
                       DeviceScratch** sc_out, StreamTables** tb_out) {
  rt_status st = validate_call(models, n_models, freq_hz, n_freq, image, params, a);
  if (st != RT_OK) return st;
  const int dev = models[0]->device;
  st = hip_check(hipSetDevice(dev), "hipSetDevice");
  if (st != RT_OK) return st;
  DeviceScratch* sc = nullptr;
  StreamTables* tb = nullptr;
  {
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    st = tables_for(dev, s, &sc, &tb);
    if (st == RT_OK) st = grow(sc, tb->launch, launch_table_bytes(a), "launch table");
    if (st == RT_OK) st = grow(sc, tb->start_ne, start_ne_bytes(a), "start n_e table");
    if (st != RT_OK) return st;
    a.launch = static_cast<const double*>(tb->launch.p);
    a.launch_ne = static_cast<const float*>(tb->start_ne.p);
  }
  st = hip_check(launch_start_index(a, static_cast<double*>(tb->launch.p), static_cast<float*>(tb->start_ne.p), s),
                 "start index");
  if (st != RT_OK) return st;
  *sc_out = sc;
  *tb_out = tb;
  return RT_OK;
}

// Enqueue the trace kernels of a call whose TraceArgs are complete except for
// the claim counters: one plain launch per image, or one persistent launch.
rt_status enqueue_trace(TraceArgs& a, const rt_params& P, int n_cu, const rt_tuning& tune, unsigned* counters,
                        hipStream_t s) {
  rt_status st = RT_OK;
  const int prec = precision_of(P.flags);
  if (P.flags & (RT_SCHED_PLAIN | RT_CARRIED_TUBE)) {
    const int waves = a.tiles_per_image;
    const int blocks = (waves + 3) / 4;
    for (int mi = 0; mi < a.n_models; ++mi)
      for (int fi = 0; fi < a.n_freq; ++fi) {
        a.image0 = mi * a.n_freq + fi;
        st = hip_check(launch_trace(a, true, prec, blocks, s), "trace launch");
        if (st != RT_OK) return st;
      }
    return RT_OK;
  }
  a.counters = counters;
  a.refill_min_idle = tune.refill_min_idle;
  const int bands = tune.xcd_bands;
  a.n_bands = bands;
  const int n_images = a.n_models * a.n_freq;
  a.range_lo[0] = 0;
  for (int x = 0; x < kXcds; ++x) {
    // rows of band x (bands = 1: every row in band 0, the others empty)
    const int row0 = x < bands ? (x * a.tiles_v) / bands : a.tiles_v;
    const int row1 = x < bands ? ((x + 1) * a.tiles_v) / bands : a.tiles_v;
    a.range_lo[x + 1] = a.range_lo[x] + (row1 - row0) * a.tiles_u * n_images;
  }
  st = hip_check(launch_fill_u32(a.counters, 0u, kXcds, s), "counter fill");
  if (st != RT_OK) return st;
  int per_cu = persistent_blocks_per_cu(prec, a.g.kind, P.flags);
  if (tune.blocks_per_cu > 0 && tune.blocks_per_cu < per_cu) per_cu = tune.blocks_per_cu;
  long long blocks = (long long)n_cu * per_cu;
  const long long max_useful = ((long long)a.range_lo[kXcds] + 3) / 4;
  if (blocks > max_useful) blocks = max_useful;
  if (blocks < 1) blocks = 1;
  return hip_check(launch_trace(a, false, prec, int(blocks), s), "persistent trace launch");
}

}  // namespace

extern "C" {

uint32_t rt_abi_version(void) { return RT_ABI_VERSION; }

const char* rt_status_string(rt_status s) {
  switch (s) {
    case RT_OK: return "RT_OK";
    case RT_E_INVALID_ARG: return "RT_E_INVALID_ARG";
    case RT_E_NONFINITE_INPUT: return "RT_E_NONFINITE_INPUT";
    case RT_E_OUT_OF_MEMORY: return "RT_E_OUT_OF_MEMORY";
    case RT_E_DEVICE: return "RT_E_DEVICE";
    case RT_E_UNSUPPORTED: return "RT_E_UNSUPPORTED";
    case RT_E_CAPACITY: return "RT_E_CAPACITY";
    case RT_E_INTERNAL: return "RT_E_INTERNAL";
  }
  return "unknown rt_status";
}

const char* rt_last_error_message(void) { return g_err.c_str(); }

rt_status rt_beam_fwhm(const double* freq_hz, int32_t n, double baseline_m, double* fwhm_out) {
  if (!freq_hz || !fwhm_out || n < 1) return fail(RT_E_INVALID_ARG, "freq_hz and fwhm_out need n >= 1 entries");
  if (!(std::isfinite(baseline_m) && baseline_m > 0.0)) return fail(RT_E_INVALID_ARG, "baseline_m must be > 0");
  const double c = 299792458.0;                     // speed of light [m/s]
  const double r_sun_over_au = 6.957e8 / 1.495978707e11;  // angle 1 R_sun subtends at 1 au [rad]
  for (int k = 0; k < n; ++k) {
    if (!(std::isfinite(freq_hz[k]) && freq_hz[k] > 0.0)) return fail(RT_E_INVALID_ARG, "frequencies must be > 0");
    fwhm_out[k] = (c / freq_hz[k] / baseline_m) / r_sun_over_au;
  }
  return RT_OK;
}

void rt_params_default(rt_params* p) {
  if (!p) return;
  std::memset(p, 0, sizeof(*p));
  p->abi_version = RT_ABI_VERSION;
  p->flags = RT_USE_MAGNIFICATION | RT_USE_REFRACTION;
  p->ds_max = 0.005;
  p->n_floor = 1.0;
  p->max_steps = 200000;
  p->checkpoint_every = 64;
  p->perturb_ratio = 1e-2;
  p->tb_inner_K = 1.0e4;
  p->tb_sky_K = 0.0;
}

rt_status rt_model_load(const rt_grid_desc* desc, const float* ne, const float* te, int32_t device, void* hip_stream,
                        rt_model** out) {
  try {
    if (!out) return fail(RT_E_INVALID_ARG, "out is NULL");
    *out = nullptr;
    rt_status st = validate_desc(desc);
    if (st != RT_OK) return st;
    if (!ne || !te) return fail(RT_E_INVALID_ARG, "ne/te is NULL");
    const long long n = (long long)desc->n0 * desc->n1 * desc->n2;
    st = validate_values_host(ne, te, n);
    if (st != RT_OK) return st;
    rt_model* m = new (std::nothrow) rt_model();
    if (!m) return fail(RT_E_OUT_OF_MEMORY, "host allocation");
    m->desc = *desc;
    m->geom = make_geom(*desc);
    m->device = device;
    const long long np = (long long)desc->n0 * desc->n1 * m->geom.n2p;
    m->nfg_bytes = size_t(np) * sizeof(float4);
    m->te_bytes = size_t(np) * sizeof(float);
    m->raw_bytes = size_t(n) * sizeof(float);
    const long long cap = byte_cap();
    if (cap >= 0 && g_device_bytes.load() + (long long)(m->nfg_bytes + m->te_bytes + 2 * m->raw_bytes) > cap) {
      delete m;
      return fail(RT_E_OUT_OF_MEMORY, "model: RT_MAX_DEVICE_BYTES exceeded");
    }
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) {
      delete m;
      return fail(RT_E_DEVICE, "no HIP device");
    }
    if (device < 0 || device >= ndev) {
      delete m;
      return fail(RT_E_INVALID_ARG, "device index out of range");
    }
    st = hip_check(hipSetDevice(device), "hipSetDevice");
    if (st == RT_OK) st = dev_alloc((void**)&m->nfg, m->nfg_bytes, "model nfg");
    if (st == RT_OK) st = dev_alloc((void**)&m->te, m->te_bytes, "model T");
    if (st == RT_OK) st = dev_alloc((void**)&m->raw_ne, m->raw_bytes, "model staging n_e");
    if (st == RT_OK) st = dev_alloc((void**)&m->raw_te, m->raw_bytes, "model staging T");
    if (st == RT_OK) st = dev_alloc((void**)&m->bad, sizeof(int), "validation counter");
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    if (st == RT_OK) st = hip_check(hipMemcpyAsync(m->raw_ne, ne, m->raw_bytes, hipMemcpyHostToDevice, s), "copy n_e");
    if (st == RT_OK) st = hip_check(hipMemcpyAsync(m->raw_te, te, m->raw_bytes, hipMemcpyHostToDevice, s), "copy T");
    if (st == RT_OK) st = stage_model(m, s);
    if (st != RT_OK) {
      free_model_memory(m);
      delete m;
      return st;
    }
    *out = m;
    return RT_OK;
  } catch (...) {
    return fail(RT_E_INTERNAL, "unexpected exception");
  }
}

rt_status rt_model_update(rt_model* m, const float* ne, const float* te, int32_t on_device, void* hip_stream) {
  try {
    if (!m) return fail(RT_E_INVALID_ARG, "model is NULL");
    if (!ne || !te) return fail(RT_E_INVALID_ARG, "ne/te is NULL");
    if (on_device < 0 || on_device > 2) return fail(RT_E_INVALID_ARG, "on_device must be 0, 1 or 2");
    const long long n = (long long)m->desc.n0 * m->desc.n1 * m->desc.n2;
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    rt_status st = hip_check(hipSetDevice(m->device), "hipSetDevice");
    if (st != RT_OK) return st;
    if (on_device == 0) {
      st = validate_values_host(ne, te, n);
      if (st != RT_OK) return st;
      st = hip_check(hipMemcpyAsync(m->raw_ne, ne, m->raw_bytes, hipMemcpyHostToDevice, s), "copy n_e");
      if (st == RT_OK) st = hip_check(hipMemcpyAsync(m->raw_te, te, m->raw_bytes, hipMemcpyHostToDevice, s), "copy T");
      if (st != RT_OK) return st;
    } else {
      // Device inputs (on_device 2: their logarithms, exponentiated into the
      // staging copies first): count invalid values with a reduction, then copy.
      if (on_device == 2) {
        st = hip_check(launch_exp_pair(ne, te, n, m->raw_ne, m->raw_te, s), "exp kernel");
        if (st != RT_OK) return st;
        ne = m->raw_ne;
        te = m->raw_te;
      }
      // (the model's own counter: no allocation, and so no device-wide
      // synchronisation of a free, in a fitting loop)
      int hbad = 0;
      st = hip_check(launch_fill_u32(reinterpret_cast<unsigned*>(m->bad), 0u, 1, s), "fill");
      if (st == RT_OK) st = hip_check(launch_validate(ne, te, n, m->bad, s), "validate kernel");
      if (st == RT_OK) st = hip_check(hipMemcpyAsync(&hbad, m->bad, sizeof(int), hipMemcpyDeviceToHost, s), "copy count");
      if (st == RT_OK) st = hip_check(hipStreamSynchronize(s), "validate sync");
      if (st != RT_OK) return st;
      if (hbad != 0)
        return fail(RT_E_NONFINITE_INPUT, std::to_string(hbad) + " model values are not finite or out of range");
      if (on_device == 1) {
        st = hip_check(hipMemcpyAsync(m->raw_ne, ne, m->raw_bytes, hipMemcpyDeviceToDevice, s), "copy n_e");
        if (st == RT_OK) st = hip_check(hipMemcpyAsync(m->raw_te, te, m->raw_bytes, hipMemcpyDeviceToDevice, s), "copy T");
        if (st != RT_OK) return st;
      }
    }
    return stage_model(m, s);
  } catch (...) {
    return fail(RT_E_INTERNAL, "unexpected exception");
  }
}

void rt_model_free(rt_model* m) {
  if (!m) return;
  if (hipSetDevice(m->device) == hipSuccess) (void)hipDeviceSynchronize();
  free_model_memory(m);
  delete m;
}

rt_status rt_trace_maps(const rt_model* const* models, int32_t n_models, const double* freq_hz, int32_t n_freq,
                        const rt_image_desc* image, const rt_params* params, float* tb_out, rt_ray_info* info_out,
                        rt_trace_stats* stats_out, const int32_t* path_rays, int32_t n_path_rays,
                        int32_t path_capacity, float* path_out, int32_t* path_len_out, void* hip_stream) {
  try {
    if (!tb_out) return fail(RT_E_INVALID_ARG, "tb_out is NULL");
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    TraceArgs a{};
    DeviceScratch* sc = nullptr;
    StreamTables* tb = nullptr;
    rt_status st = prepare_call(models, n_models, freq_hz, n_freq, image, params, s, a, &sc, &tb);
    if (st != RT_OK) return st;
    const long long total = (long long)a.nu * a.nv * n_models * n_freq;
    if (n_path_rays < 0) return fail(RT_E_INVALID_ARG, "n_path_rays < 0");
    if (n_path_rays > 0) {
      if (!path_rays || !path_out || !path_len_out || path_capacity < 1)
        return fail(RT_E_INVALID_ARG, "path outputs need path_rays, path_out, path_len_out and capacity >= 1");
      for (int k = 0; k < n_path_rays; ++k) {
        if (path_rays[k] < 0 || path_rays[k] >= total) return fail(RT_E_INVALID_ARG, "path ray index out of range");
        if (k > 0 && path_rays[k] <= path_rays[k - 1]) return fail(RT_E_INVALID_ARG, "path rays must be sorted and distinct");
      }
      {
        std::lock_guard<std::mutex> lk(g_scratch_mu);
        st = grow(sc, tb->path_rays, size_t(n_path_rays) * sizeof(int32_t), "path rays");
        if (st != RT_OK) return st;
      }
      st = hip_check(hipMemcpyAsync(tb->path_rays.p, path_rays, size_t(n_path_rays) * sizeof(int32_t),
                                    hipMemcpyHostToDevice, s), "copy path rays");
      if (st == RT_OK) st = hip_check(hipStreamSynchronize(s), "path rays sync");
      if (st != RT_OK) return st;
      a.path_rays = static_cast<const int32_t*>(tb->path_rays.p);
      a.n_path = n_path_rays;
      a.path_cap = path_capacity;
      a.path_out = path_out;
      a.path_len = path_len_out;
    }
    a.tb = tb_out;
    a.info = info_out;
    a.stats = stats_out;
    if (stats_out) {
      st = hip_check(launch_fill_u32(reinterpret_cast<unsigned*>(stats_out), 0u, sizeof(rt_trace_stats) / 4, s), "stats fill");
      if (st != RT_OK) return st;
    }
    rt_tuning tune;
    {
      std::lock_guard<std::mutex> lk(g_scratch_mu);
      tune = sc->tune;
    }
    return enqueue_trace(a, *params, sc->n_cu, tune, tb->counters, s);
  } catch (...) {
    return fail(RT_E_INTERNAL, "unexpected exception");
  }
}

rt_status rt_trace_maps_static(const rt_model* const* models, int32_t n_models, const double* freq_hz,
                               int32_t n_freq, const rt_image_desc* image, const rt_params* params, float* tb_out,
                               rt_ray_info* info_out, rt_trace_stats* stats_out, void* hip_stream) {
  try {
    if (!tb_out) return fail(RT_E_INVALID_ARG, "tb_out is NULL");
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    TraceArgs a{};
    rt_status st = validate_call(models, n_models, freq_hz, n_freq, image, params, a);
    if (st != RT_OK) return st;
    const size_t lt = (launch_table_bytes(a) + 255) / 256 * 256;
    const size_t ne = start_ne_bytes(a);
    if (kStaticCountersBytes + lt + ne > kStaticScratchBytes)
      return fail(RT_E_CAPACITY, "rt_trace_maps_static: the call needs " +
                                     std::to_string(kStaticCountersBytes + lt + ne) + " bytes of scratch, more than " +
                                     std::to_string(kStaticScratchBytes) + " (nu*nv*(48 + 4*n_models) + 256)");
    const int dev = models[0]->device;
    st = hip_check(hipSetDevice(dev), "hipSetDevice");
    if (st != RT_OK) return st;
    DeviceScratch* sc = nullptr;
    rt_tuning tune;
    char* base = nullptr;
    {
      std::lock_guard<std::mutex> lk(g_scratch_mu);
      st = scratch_for(dev, &sc);
      if (st != RT_OK) return st;
      if (!g_static_ptr[dev]) {
        void* ptr = nullptr;
        st = hip_check(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)), "hipGetSymbolAddress(scratch)");
        if (st != RT_OK) return st;
        g_static_ptr[dev] = ptr;
      }
      base = static_cast<char*>(g_static_ptr[dev]);
      tune = sc->tune;
    }
    unsigned* counters = reinterpret_cast<unsigned*>(base);
    double* launch = reinterpret_cast<double*>(base + kStaticCountersBytes);
    float* start_ne = reinterpret_cast<float*>(base + kStaticCountersBytes + lt);
    a.launch = launch;
    a.launch_ne = start_ne;
    st = hip_check(launch_start_index(a, launch, start_ne, s), "start index");
    if (st != RT_OK) return st;
    a.tb = tb_out;
    a.info = info_out;
    a.stats = stats_out;
    if (stats_out) {
      st = hip_check(launch_fill_u32(reinterpret_cast<unsigned*>(stats_out), 0u, sizeof(rt_trace_stats) / 4, s), "stats fill");
      if (st != RT_OK) return st;
    }
    return enqueue_trace(a, *params, sc->n_cu, tune, counters, s);
  } catch (...) {
    return fail(RT_E_INTERNAL, "unexpected exception");
  }
}

void rt_tuning_default(rt_tuning* t) {
  if (!t) return;
  t->abi_version = RT_ABI_VERSION;
  t->refill_min_idle = 64;
  t->blocks_per_cu = 0;
  t->xcd_bands = kXcds;
}

rt_status rt_set_tuning(int device, const rt_tuning* t) {
  try {
    if (!t) return fail(RT_E_INVALID_ARG, "tuning is NULL");
    if (t->abi_version != RT_ABI_VERSION) return fail(RT_E_INVALID_ARG, "tuning->abi_version mismatch");
    if (t->refill_min_idle < 1 || t->refill_min_idle > 64) return fail(RT_E_INVALID_ARG, "refill_min_idle must be 1..64");
    if (t->blocks_per_cu < 0 || t->blocks_per_cu > 8) return fail(RT_E_INVALID_ARG, "blocks_per_cu must be 0..8");
    if (t->xcd_bands != 1 && t->xcd_bands != kXcds) return fail(RT_E_INVALID_ARG, "xcd_bands must be 1 or 8");
    DeviceScratch* sc = nullptr;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    rt_status st = scratch_for(device, &sc);
    if (st != RT_OK) return st;
    sc->tune = *t;
    return RT_OK;
  } catch (...) {
    return fail(RT_E_INTERNAL, "unexpected exception");
  }
}

rt_status rt_get_tuning(int device, rt_tuning* t) {
  try {
    if (!t) return fail(RT_E_INVALID_ARG, "tuning is NULL");
    DeviceScratch* sc = nullptr;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    rt_status st = scratch_for(device, &sc);
    if (st != RT_OK) return st;
    *t = sc->tune;
    return RT_OK;
  } catch (...) {
    return fail(RT_E_INTERNAL, "unexpected exception");
  }
}

rt_status rt_autotune(const rt_model* const* models, int32_t n_models, const double* freq_hz, int32_t n_freq,
                      const rt_image_desc* image, const rt_params* params, int32_t max_freqs, rt_tuning* best,
                      double* best_ms, double* default_ms, void* hip_stream) {
  try {
    if (max_freqs < 1) return fail(RT_E_INVALID_ARG, "max_freqs must be >= 1");
    if (!models || n_models < 1 || !models[0]) return fail(RT_E_INVALID_ARG, "need at least one model");
    if (!freq_hz || n_freq < 1) return fail(RT_E_INVALID_ARG, "need at least one frequency");
    if (!image || !params) return fail(RT_E_INVALID_ARG, "image/params is NULL");
    if (params->flags & (RT_SCHED_PLAIN | RT_CARRIED_TUBE))
      return fail(RT_E_INVALID_ARG, "the tuning applies to the persistent trace");
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    const int dev = models[0]->device;
    rt_status st = hip_check(hipSetDevice(dev), "hipSetDevice");
    if (st != RT_OK) return st;
    DeviceScratch* sc = nullptr;
    rt_tuning saved;
    {
      std::lock_guard<std::mutex> lk(g_scratch_mu);
      st = scratch_for(dev, &sc);
      if (st != RT_OK) return st;
      saved = sc->tune;
    }
    // the sample: at most max_freqs frequencies spread over the list
    const int m = std::min<int>(max_freqs, n_freq);
    std::vector<double> fs(m);
    for (int k = 0; k < m; ++k) fs[k] = freq_hz[int(((long long)(2 * k + 1) * n_freq) / (2 * m))];
    const long long n_out = (long long)n_models * m * image->nu * image->nv;
    if (n_out < 1 || n_out > (1ll << 31) - 1) return fail(RT_E_CAPACITY, "sample too large");
    float* ref = nullptr;
    float* cur = nullptr;
    unsigned* diff = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    auto cleanup = [&]() {
      if (e0) (void)hipEventDestroy(e0);
      if (e1) (void)hipEventDestroy(e1);
      dev_free(ref, size_t(n_out) * sizeof(float));
      dev_free(cur, size_t(n_out) * sizeof(float));
      dev_free(diff, sizeof(unsigned));
      std::lock_guard<std::mutex> lk(g_scratch_mu);
      sc->tune = saved;
    };
    st = dev_alloc((void**)&ref, size_t(n_out) * sizeof(float), "autotune maps");
    if (st == RT_OK) st = dev_alloc((void**)&cur, size_t(n_out) * sizeof(float), "autotune maps");
    if (st == RT_OK) st = dev_alloc((void**)&diff, sizeof(unsigned), "autotune counter");
    if (st == RT_OK) st = hip_check(hipEventCreate(&e0), "event");
    if (st == RT_OK) st = hip_check(hipEventCreate(&e1), "event");
    if (st != RT_OK) { cleanup(); return st; }
    const int max_per_cu = persistent_blocks_per_cu(precision_of(params->flags), models[0]->geom.kind, params->flags);
    std::vector<rt_tuning> cand;
    rt_tuning d;
    rt_tuning_default(&d);
    cand.push_back(d);  // the defaults first: the reference maps
    const int refills[5] = {64, 32, 16, 8, 1};
    for (int bands : {int(kXcds), 1})
      for (int bpc = 1; bpc <= max_per_cu; ++bpc)
        for (int rf : refills) {
          rt_tuning t = d;
          t.refill_min_idle = rf;
          t.blocks_per_cu = bpc;
          t.xcd_bands = bands;
          if (!(bands == d.xcd_bands && rf == d.refill_min_idle && bpc == max_per_cu)) cand.push_back(t);
        }
    auto run = [&](const rt_tuning& t, float* out, double* ms) -> rt_status {
      {
        std::lock_guard<std::mutex> lk(g_scratch_mu);
        sc->tune = t;
      }
      rt_status r = hip_check(hipEventRecord(e0, s), "event record");
      if (r == RT_OK)
        r = rt_trace_maps(models, n_models, fs.data(), m, image, params, out, nullptr, nullptr, nullptr, 0, 0,
                          nullptr, nullptr, hip_stream);
      if (r == RT_OK) r = hip_check(hipEventRecord(e1, s), "event record");
      if (r == RT_OK) r = hip_check(hipEventSynchronize(e1), "event sync");
      float f = 0.f;
      if (r == RT_OK) r = hip_check(hipEventElapsedTime(&f, e0, e1), "event time");
      *ms = double(f);
      return r;
    };
    double ms = 0.0;
    st = run(cand[0], ref, &ms);  // warm-up (first use of the model and the launch table)
    if (st == RT_OK) st = run(cand[0], ref, &ms);
    const double ms_default = ms;
    rt_tuning chosen = cand[0];
    double ms_best = ms;
    for (size_t k = 1; st == RT_OK && k < cand.size(); ++k) {
      st = run(cand[k], cur, &ms);
      if (st != RT_OK) break;
      unsigned nd = 0;
      st = hip_check(launch_fill_u32(diff, 0u, 1, s), "diff fill");
      if (st == RT_OK) st = hip_check(launch_count_diff(reinterpret_cast<const unsigned*>(ref),
                                                        reinterpret_cast<const unsigned*>(cur), n_out, diff, s),
                                      "map compare");
      if (st == RT_OK) st = hip_check(hipMemcpyAsync(&nd, diff, sizeof(unsigned), hipMemcpyDeviceToHost, s), "copy");
      if (st == RT_OK) st = hip_check(hipStreamSynchronize(s), "stream sync");
      if (st != RT_OK) break;
      if (nd != 0) {
        cleanup();
        return fail(RT_E_INTERNAL, "autotune: maps differ between launch tunings");
      }
      if (ms < ms_best) { ms_best = ms; chosen = cand[k]; }
    }
    cleanup();
    if (st != RT_OK) return st;
    {
      std::lock_guard<std::mutex> lk(g_scratch_mu);
      sc->tune = chosen;
    }
    if (best) *best = chosen;
    if (best_ms) *best_ms = ms_best;
    if (default_ms) *default_ms = ms_default;
    return RT_OK;
  } catch (...) {
    return fail(RT_E_INTERNAL, "unexpected exception");
  }
}

rt_status rt_beam_convolve(const float* maps_in, float* maps_out, int32_t n_maps, int32_t nu, int32_t nv,
                           double half_u, double half_v, const double* fwhm, void* hip_stream) {
  try {
    if (!maps_in || !maps_out || !fwhm) return fail(RT_E_INVALID_ARG, "maps_in, maps_out and fwhm must not be NULL");
    if (maps_in == maps_out) return fail(RT_E_INVALID_ARG, "maps_out must not alias maps_in");
    if (n_maps < 1 || n_maps > kMaxBlurMaps) return fail(RT_E_INVALID_ARG, "n_maps must be 1..128");
    if (nu < 1 || nv < 1) return fail(RT_E_INVALID_ARG, "nu, nv must be >= 1");
    if (!(std::isfinite(half_u) && std::isfinite(half_v) && half_u > 0 && half_v > 0))
      return fail(RT_E_INVALID_ARG, "half widths must be finite and > 0");
    if ((long long)nu * nv * n_maps > (1ll << 31) - 1) return fail(RT_E_CAPACITY, "more than 2^31-1 pixels");
    BlurArgs b{};
    b.n_maps = n_maps; b.nu = nu; b.nv = nv;
    const double pix[2] = {2.0 * half_u / nu, 2.0 * half_v / nv};
    for (int m = 0; m < n_maps; ++m) {
      if (!(std::isfinite(fwhm[m]) && fwhm[m] >= 0.0)) return fail(RT_E_INVALID_ARG, "fwhm must be finite and >= 0");
      for (int ax = 0; ax < 2; ++ax) {
        const double sigma = fwhm[m] / (2.0 * std::sqrt(2.0 * std::log(2.0))) / pix[ax];  // in pixels
        const int len = ax == 0 ? nu : nv;
        int R = sigma > 0.0 ? int(std::ceil(5.0 * sigma)) : 0;
        if (R > len - 1) R = len - 1;
        const double c = sigma > 0.0 ? 1.0 / (2.0 * sigma * sigma) : 0.0;
        double norm = 0.0;
        for (int k = -R; k <= R; ++k) norm += std::exp(-double(k) * k * c);
        (ax == 0 ? b.radius_u : b.radius_v)[m] = R;
        (ax == 0 ? b.inv2s2_u : b.inv2s2_v)[m] = float(c);
        (ax == 0 ? b.inv_norm_u : b.inv_norm_v)[m] = float(1.0 / norm);
      }
    }
    int dev = 0;
    rt_status st = hip_check(hipGetDevice(&dev), "hipGetDevice");
    if (st != RT_OK) return st;
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    const size_t bytes = size_t(nu) * nv * n_maps * sizeof(float);
    float* tmp = nullptr;
    {
      std::lock_guard<std::mutex> lk(g_scratch_mu);
      DeviceScratch* sc = nullptr;
      StreamTables* tb = nullptr;
      st = tables_for(dev, s, &sc, &tb);
      if (st == RT_OK) st = grow(sc, tb->blur_tmp, bytes, "beam scratch");
      if (st != RT_OK) return st;
      tmp = static_cast<float*>(tb->blur_tmp.p);
    }
    return hip_check(launch_blur(b, maps_in, tmp, maps_out, s), "beam convolution");
  } catch (...) {
    return fail(RT_E_INTERNAL, "unexpected exception");
  }
}

rt_status rt_disc_mean(const float* maps, int32_t n_maps, int32_t nu, int32_t nv, double half_u, double half_v,
                       double radius, double* mean_out, void* hip_stream) {
  try {
    if (!maps || !mean_out) return fail(RT_E_INVALID_ARG, "maps and mean_out must not be NULL");
    if (n_maps < 1 || nu < 1 || nv < 1) return fail(RT_E_INVALID_ARG, "n_maps, nu, nv must be >= 1");
    if (!(std::isfinite(half_u) && std::isfinite(half_v) && half_u > 0 && half_v > 0))
      return fail(RT_E_INVALID_ARG, "half widths must be finite and > 0");
    if (!(std::isfinite(radius) && radius > 0)) return fail(RT_E_INVALID_ARG, "radius must be finite and > 0");
    if ((long long)nu * nv * n_maps > (1ll << 31) - 1) return fail(RT_E_CAPACITY, "more than 2^31-1 pixels");
    DiscArgs d{};
    d.n_maps = n_maps; d.nu = nu; d.nv = nv;
    d.half_u = half_u; d.half_v = half_v;
    d.pix_u = 2.0 * half_u / nu; d.pix_v = 2.0 * half_v / nv;
    d.radius2 = radius * radius;
    return hip_check(launch_disc_mean(d, maps, mean_out, static_cast<hipStream_t>(hip_stream)), "disc mean");
  } catch (...) {
    return fail(RT_E_INTERNAL, "unexpected exception");
  }
}

rt_status rt_probe_read_bandwidth(int32_t device, int64_t bytes, int64_t span_bytes, int32_t blocks, int32_t reps,
                                  double* gbps_out, void* hip_stream) {
  try {
    if (!gbps_out) return fail(RT_E_INVALID_ARG, "gbps_out is NULL");
    if (bytes < 16 || bytes % 16 != 0) return fail(RT_E_INVALID_ARG, "bytes must be a positive multiple of 16");
    if (span_bytes < 16 || span_bytes % 16 != 0 || span_bytes > bytes)
      return fail(RT_E_INVALID_ARG, "span_bytes must be a multiple of 16 in [16, bytes]");
    if (blocks < 1 || blocks > (1 << 20)) return fail(RT_E_INVALID_ARG, "blocks must be in [1, 2^20]");
    if (reps < 1 || reps > 4096) return fail(RT_E_INVALID_ARG, "reps must be in [1, 4096]");
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    rt_status st = hip_check(hipSetDevice(device), "hipSetDevice");
    if (st != RT_OK) return st;
    float4* buf = nullptr;
    float* sink = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    const size_t sink_bytes = size_t(blocks) * 256 * sizeof(float);
    auto cleanup = [&]() {
      if (e0) (void)hipEventDestroy(e0);
      if (e1) (void)hipEventDestroy(e1);
      dev_free(buf, size_t(bytes));
      dev_free(sink, sink_bytes);
    };
    st = dev_alloc((void**)&buf, size_t(bytes), "probe buffer");
    if (st == RT_OK) st = dev_alloc((void**)&sink, sink_bytes, "probe sink");
    if (st == RT_OK) st = hip_check(hipMemsetAsync(buf, 0, size_t(bytes), s), "probe fill");
    if (st == RT_OK) st = hip_check(hipEventCreate(&e0), "event");
    if (st == RT_OK) st = hip_check(hipEventCreate(&e1), "event");
    const long long n4 = bytes / 16, span4 = span_bytes / 16;
    // one untimed launch, then the timed one
    if (st == RT_OK) st = hip_check(launch_stream_read(buf, n4, span4, blocks, reps, sink, s), "probe launch");
    if (st == RT_OK) st = hip_check(hipEventRecord(e0, s), "event record");
    if (st == RT_OK) st = hip_check(launch_stream_read(buf, n4, span4, blocks, reps, sink, s), "probe launch");
    if (st == RT_OK) st = hip_check(hipEventRecord(e1, s), "event record");
    if (st == RT_OK) st = hip_check(hipEventSynchronize(e1), "event sync");
    float ms = 0.f;
    if (st == RT_OK) st = hip_check(hipEventElapsedTime(&ms, e0, e1), "elapsed");
    if (st == RT_OK) {
      if (!(ms > 0.f)) st = fail(RT_E_DEVICE, "probe time not positive");
      else *gbps_out = double(span_bytes) * double(blocks) * double(reps) / (double(ms) * 1e-3) * 1e-9;
    }
    cleanup();
    return st;
  } catch (...) {
    return fail(RT_E_INTERNAL, "unexpected exception");
  }
}

rt_status rt_probe_path_keys(const rt_model* model, const float* path, const int32_t* path_len, int32_t n_walks,
                             int32_t path_capacity, int32_t* keys_out, void* hip_stream) {
  try {
    if (!model || !path || !path_len || !keys_out) return fail(RT_E_INVALID_ARG, "NULL argument");
    if (n_walks < 1 || path_capacity < 1) return fail(RT_E_INVALID_ARG, "n_walks and path_capacity must be >= 1");
    if ((long long)n_walks * path_capacity > (1ll << 31) - 1) return fail(RT_E_CAPACITY, "more than 2^31-1 keys");
    rt_status st = hip_check(hipSetDevice(model->device), "hipSetDevice");
    if (st != RT_OK) return st;
    return hip_check(launch_path_keys(model->geom, path, path_len, n_walks, path_capacity, keys_out,
                                      static_cast<hipStream_t>(hip_stream)),
                     "path keys");
  } catch (...) {
    return fail(RT_E_INTERNAL, "unexpected exception");
  }
}

rt_status rt_probe_gather_replay(const rt_model* model, const int32_t* keys, int32_t n_walks, int32_t path_capacity,
                                 double* ms_out, void* hip_stream) {
  try {
    if (!model || !keys || !ms_out) return fail(RT_E_INVALID_ARG, "NULL argument");
    if (n_walks < 1 || path_capacity < 1) return fail(RT_E_INVALID_ARG, "n_walks and path_capacity must be >= 1");
    if ((long long)n_walks * path_capacity > (1ll << 31) - 1) return fail(RT_E_CAPACITY, "more than 2^31-1 keys");
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    rt_status st = hip_check(hipSetDevice(model->device), "hipSetDevice");
    if (st != RT_OK) return st;
    const DevGeom& g = model->geom;
    const int s1 = g.n2p, s0 = g.n1 * g.n2p;
    const long long n_vert = (long long)g.n0 * s0;
    const long long mk = n_vert - 1 - (s0 + s1 + 1);
    if (mk < 0) return fail(RT_E_INVALID_ARG, "grid too small");
    const int max_key = int(std::min<long long>(mk, (1ll << 31) - 1));
    float* sink = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    const size_t sink_bytes = size_t(n_walks) * sizeof(float);
    auto cleanup = [&]() {
      if (e0) (void)hipEventDestroy(e0);
      if (e1) (void)hipEventDestroy(e1);
      dev_free(sink, sink_bytes);
    };
    st = dev_alloc((void**)&sink, sink_bytes, "replay sink");
    if (st == RT_OK) st = hip_check(hipEventCreate(&e0), "event");
    if (st == RT_OK) st = hip_check(hipEventCreate(&e1), "event");
    auto launch = [&]() {
      return hip_check(launch_gather_replay(model->nfg, model->te, keys, n_walks, path_capacity, s0, s1, max_key, sink, s),
                       "replay launch");
    };
    if (st == RT_OK) st = launch();
    if (st == RT_OK) st = hip_check(hipEventRecord(e0, s), "event record");
    if (st == RT_OK) st = launch();
    if (st == RT_OK) st = hip_check(hipEventRecord(e1, s), "event record");
    if (st == RT_OK) st = hip_check(hipEventSynchronize(e1), "event sync");
    float ms = 0.f;
    if (st == RT_OK) st = hip_check(hipEventElapsedTime(&ms, e0, e1), "elapsed");
    if (st == RT_OK) *ms_out = double(ms);
    cleanup();
    return st;
  } catch (...) {
    return fail(RT_E_INTERNAL, "unexpected exception");
  }
}

rt_status rt_trace_adjoint(const rt_model* model, const double* freq_hz, int32_t n_freq, const rt_image_desc* image,
                           const rt_params* params, const float* weights, double* loss_out, float* grad_ln_ne,
                           float* grad_ln_te, float* tb_out, void* hip_stream) {
  try {
    if (!model) return fail(RT_E_INVALID_ARG, "model is NULL");
    if (!weights || !loss_out || !grad_ln_ne || !grad_ln_te)
      return fail(RT_E_INVALID_ARG, "weights, loss_out, grad_ln_ne and grad_ln_te must not be NULL");
    if (params && (params->flags & (RT_PREC_ALL_FP32 | RT_PREC_FP32_STEP)))
      return fail(RT_E_UNSUPPORTED, "the adjoint runs in the default precision only");
    if (params && (params->flags & RT_TEST_NO_ABSORPTION))
      return fail(RT_E_UNSUPPORTED, "RT_TEST_NO_ABSORPTION is a forward-only test mode");
    if (params && (params->flags & RT_DETERMINISTIC_GRAD))
      return fail(RT_E_UNSUPPORTED, "RT_DETERMINISTIC_GRAD is not supported by this build");
    if (params && (params->flags & RT_CARRIED_TUBE))
      return fail(RT_E_UNSUPPORTED, "the adjoint differentiates the step-wise tube estimate only");
    if (params && params->checkpoint_every < 0) return fail(RT_E_INVALID_ARG, "checkpoint_every must be >= 0");
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    // The workspace is sized per call and may be reallocated: a captured graph
    // would keep a pointer to freed memory, so capture is refused.
    hipStreamCaptureStatus cap_status = hipStreamCaptureStatusNone;
    rt_status st = hip_check(hipStreamIsCapturing(s, &cap_status), "hipStreamIsCapturing");
    if (st != RT_OK) return st;
    if (cap_status != hipStreamCaptureStatusNone)
      return fail(RT_E_UNSUPPORTED, "rt_trace_adjoint cannot be captured in a graph");
    TraceArgs a{};
    DeviceScratch* sc = nullptr;
    StreamTables* tbl = nullptr;
    const rt_model* models[1] = {model};
    st = prepare_call(models, 1, freq_hz, n_freq, image, params, s, a, &sc, &tbl);
    if (st != RT_OK) return st;
    const rt_params& P = *params;
    const long long npx = (long long)a.nu * a.nv;
    const int K = P.checkpoint_every > 0 ? P.checkpoint_every : 64;
    long long cap = ((long long)P.max_steps + K - 1) / K + 1;
    if (cap > kAdjMaxCheckpoints) cap = kAdjMaxCheckpoints;
    if (cap < 2) cap = 2;
    cap += cap & 1;  // even: thinning keeps every other checkpoint
    const int n_tiles = a.tiles_per_image * n_freq;
    // checkpoints are kept per ray: the tiles are traced and swept in batches
    // whose checkpoints fit the budget
    const long long tile_bytes = (long long)kWaveLanes * (cap * kCkptFields * (long long)sizeof(double) + 3 * 4);
    const long long budget = env_bytes("RT_ADJOINT_CHECKPOINT_BYTES");
    long long batch = (budget > 0 ? budget : kAdjCheckpointBudget) / tile_bytes;
    if (batch < 1) batch = 1;
    if (batch > n_tiles) batch = n_tiles;
    long long blocks = (long long)sc->n_cu * adjoint_blocks_per_cu(a.g.kind);
    const long long max_useful = (batch + 3) / 4;
    if (blocks > max_useful) blocks = max_useful;
    if (blocks < 1) blocks = 1;
    const long long n_slots = blocks * 256;
    const long long n_rays = batch * kWaveLanes;
    const size_t ck_bytes = size_t(cap) * kCkptFields * size_t(n_rays) * sizeof(double);
    const size_t meta_bytes = size_t(3) * size_t(n_rays) * sizeof(int);
    const size_t st_bytes = size_t(K) * kCkptFields * size_t(n_slots) * sizeof(double);
    const size_t tp_bytes = size_t(K) * kTapeFields * size_t(n_slots) * sizeof(float);
    const long long nvp = (long long)a.g.n0 * a.g.n1 * a.g.n2p;
    const size_t acc_bytes = size_t(nvp) * kGradChannels * sizeof(double);
    const size_t tb_bytes = tb_out ? 0 : size_t(npx) * size_t(n_freq) * sizeof(float);
    const size_t need = ck_bytes + meta_bytes + st_bytes + tp_bytes + acc_bytes + tb_bytes + 256 * 4;
    char* ws = nullptr;
    {
      std::lock_guard<std::mutex> lk(g_scratch_mu);
      st = grow(sc, tbl->adj, need, "adjoint workspace", /*can_free=*/true);
      if (st != RT_OK) return st;
      ws = static_cast<char*>(tbl->adj.p);
    }
    AdjointArgs aa{};
    size_t off = 0;
    aa.gacc = reinterpret_cast<double*>(ws + off); off += acc_bytes;
    aa.ckpt = reinterpret_cast<double*>(ws + off); off += ck_bytes;
    aa.steps = reinterpret_cast<double*>(ws + off); off += st_bytes;
    aa.tape = reinterpret_cast<float*>(ws + off); off += tp_bytes;
    aa.meta = reinterpret_cast<int*>(ws + off); off += (meta_bytes + 255) / 256 * 256;
    float* tb = tb_out ? tb_out : reinterpret_cast<float*>(ws + off);
    a.tb = tb;
    a.info = nullptr;
    a.stats = nullptr;
    aa.t = a;
    aa.weights = weights;
    aa.loss = loss_out;
    aa.K = K;
    aa.ckpt_cap = int(cap);
    aa.n_slots = int(n_slots);
    st = hip_check(launch_fill_u32(reinterpret_cast<unsigned*>(aa.gacc), 0u, (long long)(acc_bytes / 4), s), "gradient fill");
    if (st == RT_OK) st = hip_check(launch_fill_u32(reinterpret_cast<unsigned*>(loss_out), 0u, 2, s), "loss fill");
    for (int t0 = 0; st == RT_OK && t0 < n_tiles; t0 += int(batch)) {
      aa.tile0 = t0;
      aa.n_tiles = int(std::min<long long>(batch, n_tiles - t0));
      aa.n_rays = aa.n_tiles * kWaveLanes;
      aa.counter = tbl->counters;
      st = hip_check(launch_fill_u32(aa.counter, 0u, 1, s), "counter fill");
      if (st == RT_OK) st = hip_check(launch_adjoint_forward(aa, s), "adjoint forward launch");
      if (st == RT_OK) st = hip_check(launch_adjoint(aa, int(blocks), s), "adjoint launch");
    }
    if (st == RT_OK)
      st = hip_check(launch_unpack_grad(a.g, model->nfg, model->te, aa.gacc, grad_ln_ne, grad_ln_te, s), "gradient gather");
    return st;
  } catch (...) {
    return fail(RT_E_INTERNAL, "unexpected exception");
  }
}

}  // extern "C"
