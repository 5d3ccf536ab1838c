// vqs_host.cpp -- host runtime of the library: argument checks, per-stream workspaces,
// the level loop of the breadth-first recursion, hipGraph capture for segmented
// sorts, statistics, and the C interface declared in include/vqs.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cstdio>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <tuple>
#include <vector>

#include "../../include/vqs.h"
#include "vqs_launch.h"
#include "vqs_learned.h"
#include "vqs_stable.h"

// Fixed device scratch of vqs_sort_noalloc: every device the library runs on holds its
// own copy from the library's load until the process ends.  In host code this name
// stands for a host-side shadow, not a device address: each device's address comes
// from hipGetSymbolAddress (noalloc_setup) and only that address is used.
static __device__ __align__(256) unsigned char scratch[VQS_NOALLOC_SCRATCH_BYTES];

namespace vqs {

namespace {

constexpr int VERSION = 10000;  // 1.0.0

struct Geometry {
  int num_cu = 256;
  int level_grid = 2048;
  int solo_grid = 512;
  int pivot_grid = 256;
  int plan_grid = 512;
};

struct GraphKey {
  const void* ws_base;   // workspace the graph's launches use
  void* keys;
  const int64_t* offsets;
  uint64_t nseg, n;
  int kt, asc;
  uint64_t seed;
  int64_t depth_limit, fb_limit;
  uint32_t nb, local;
  uint64_t solo;
  int run_mode, tile;
  uint32_t rng_mode;
  std::array<uint32_t, 8> rng_key;
  int inplace;
  bool operator<(const GraphKey& o) const {
    return std::tie(ws_base, keys, offsets, nseg, n, kt, asc, seed, depth_limit, fb_limit, nb, local, solo,
                    run_mode, tile, rng_mode, rng_key, inplace) <
           std::tie(o.ws_base, o.keys, o.offsets, o.nseg, o.n, o.kt, o.asc, o.seed, o.depth_limit, o.fb_limit, o.nb,
                    o.local, o.solo, o.run_mode, o.tile, o.rng_mode, o.rng_key, o.inplace);
  }
};

struct ProfRec {
  int kind, level;
  hipEvent_t a, b;
};

int g_profile = 0;   // vqs_profile: 0 off, 1 every launch, 2 level partitions only

struct Workspace {
  int device = 0;
  hipStream_t stream = nullptr;
  char* mem = nullptr;
  size_t bytes = 0;
  // capacities the allocation was carved for
  uint64_t cap_n = 0, cap_lvl = 0, cap_tiles = 0, cap_solo = 0, cap_scratch_bytes = 0;
  uint64_t cap_ip_stash = 0, cap_ip_pfx = 0;
  int cap_levels = 0;
  Params p{};  // carved pointers
  unsigned long long* host_pinned = nullptr;
  unsigned long long host_word[8] = {};   // pageable stand-in when host_pinned is absent
  unsigned long long* ctr_word() { return host_pinned ? host_pinned : host_word; }
  int p_levels = 0;          // level counters p.lvl_ctr holds
  bool p_external = false;   // p points into a caller's workspace, not into mem
  int last_levels = 0;
  bool have_result = false;
  // learned splitter buffers
  char* lmem = nullptr;
  uint64_t lcap_m = 0, lcap_chunks = 0;
  uint64_t* l_sample = nullptr;
  float* l_x = nullptr;
  float* l_t = nullptr;
  float* l_params = nullptr;
  float* l_moments = nullptr;
  uint64_t* l_thr = nullptr;
  uint32_t* l_nvalid = nullptr;
  uint32_t* l_hist = nullptr;
  uint64_t* l_totals = nullptr;
  int64_t* l_offsets = nullptr;
  uint64_t* l_summary = nullptr;
  bool learned_ran = false;
  char* smem = nullptr;   // stable sort: the composite keys
  size_t scap = 0;
  std::unique_ptr<Workspace> inner;  // for sorting the sample
  hipGraphExec_t graph = nullptr;
  GraphKey graph_key{};
  bool graph_valid = false;
  std::vector<hipEvent_t> event_pool;
  std::vector<ProfRec> prof;
  size_t events_used = 0;
  bool capturing = false;
  bool owned = true;       // false: mem belongs to someone else (nothing freed)
  bool no_profile = false; // never record profiling events (the allocation-free path)
  uint64_t seq = 0;        // order of the calls that left a result (newest is largest)
  hipEvent_t next_event() {
    if (events_used == event_pool.size()) {
      hipEvent_t e = nullptr;
      if (hipEventCreate(&e) != hipSuccess) return nullptr;
      event_pool.push_back(e);
    }
    return event_pool[events_used++];
  }
  // record an event pair around a launch when profiling
  template <class F>
  hipError_t timed(int kind, int level, F&& launch) {
    if (!g_profile || (g_profile == 2 && kind != 2) || capturing || no_profile) return launch();
    hipEvent_t a = next_event(), b = next_event();
    if (a) (void)hipEventRecord(a, stream);
    hipError_t e = launch();
    if (b) (void)hipEventRecord(b, stream);
    if (a && b) prof.push_back(ProfRec{kind, level, a, b});
    return e;
  }
  ~Workspace() {
    for (hipEvent_t e : event_pool) (void)hipEventDestroy(e);
    if (graph) (void)hipGraphExecDestroy(graph);
    if (!owned) return;
    if (mem) (void)hipFree(mem);
    if (host_pinned) (void)hipHostFree(host_pinned);
    if (lmem) (void)hipFree(lmem);
    if (smem) (void)hipFree(smem);
  }
};

std::mutex g_mu;
std::map<std::pair<int, hipStream_t>, std::unique_ptr<Workspace>> g_ws;
uint64_t g_seq = 0;  // numbers the calls that leave a result
std::map<int, Geometry> g_geom;

Geometry geometry_of(int dev) {
  Geometry g;
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, dev) == hipSuccess && prop.multiProcessorCount > 0)
    g.num_cu = prop.multiProcessorCount;
  else
    (void)hipGetLastError();
  g.level_grid = g.num_cu * 8;
  g.solo_grid = g.num_cu * (1024 / SOLO_P);   // the solo kernel's LDS and registers allow 1024 threads per CU
  g.plan_grid = g.num_cu * 2;
  return g;
}

Geometry geometry(int dev) {
  auto it = g_geom.find(dev);
  if (it != g_geom.end()) return it->second;
  const Geometry g = geometry_of(dev);
  g_geom[dev] = g;
  return g;
}

int key_bits(int kt) {
  switch (kt) {
    case VQS_U16: case VQS_I16: return 16;
    case VQS_U32: case VQS_F32: case VQS_I32: return 32;
    case VQS_U64: case VQS_F64: case VQS_I64: return 64;
    case VQS_U128: case VQS_K64V64: return 128;
    default: return 0;
  }
}

uint64_t level_tile_keys(int bits, int tile) {
  switch (bits) {
    case 16: return tile ? LaunchLevel<16, level_chunks_half(16)>::level_tile_keys()
                         : LaunchLevel<16, level_chunks(16)>::level_tile_keys();
    case 32: return tile ? LaunchLevel<32, level_chunks_half(32)>::level_tile_keys()
                         : LaunchLevel<32, level_chunks(32)>::level_tile_keys();
    case 64: return tile ? LaunchLevel<64, level_chunks_half(64)>::level_tile_keys()
                         : LaunchLevel<64, level_chunks(64)>::level_tile_keys();
    default: return tile ? LaunchLevel<128, level_chunks_half(128)>::level_tile_keys()
                         : LaunchLevel<128, level_chunks(128)>::level_tile_keys();
  }
}

uint64_t local_buffer_keys(int bits) {
  switch (bits) {
    case 16: return Launch<16>::local_buffer_keys();
    case 32: return Launch<32>::local_buffer_keys();
    case 64: return Launch<64>::local_buffer_keys();
    default: return Launch<128>::local_buffer_keys();
  }
}

uint32_t depth_limit_for(uint64_t n) {
  uint32_t lg = 0;
  while ((n >> (lg + 1)) != 0) lg++;
  return 2 * lg + 4;
}

// True when the caller's options structure holds the field ending at byte `end`
// (struct_size 0 is taken as the full structure).
bool has_field(const vqs_options* o, size_t end) { return o && (o->struct_size == 0 || o->struct_size >= end); }
#define VQS_HAS(o, f) has_field((o), offsetof(vqs_options, f) + sizeof(((vqs_options*)0)->f))

// Transform of the caller's keys into the internal ascending unsigned form.
int mode_of(int kt, int asc) {
  return ((kt == VQS_F32 || kt == VQS_F64) ? MODE_FLOAT : 0) |
         ((kt == VQS_I16 || kt == VQS_I32 || kt == VQS_I64) ? MODE_SIGNED : 0) | (asc ? 0 : MODE_DESC);
}

struct Plan {
  int bits, ks, mode;
  uint64_t n, nseg;
  uint32_t nb, local;
  uint64_t solo;
  int max_levels;
  uint64_t cap_lvl, cap_tiles, cap_solo;
  uint64_t seed;
  int64_t depth_limit;  // < 0: default per range, else this limit for every range
  int64_t fb_limit;     // < 0: default per range, else the fallback mode's own limit
  int run_mode;         // level partitions write tile-local runs
  int tile;             // level tile size: 0 default, 1 half
  uint32_t rng_mode;    // pivot sampler: 0 SFC64, 1 ChaCha20
  uint32_t rng_key[8];
  int inplace;          // in-place partitions, no key scratch
  uint32_t ip_steps;    // in-place level tiles: loop blocks per tile
};

int make_plan(uint64_t n, uint64_t nseg, int kt, int asc, const vqs_options* o, const Geometry& g, Plan* pl) {
  const int bits = key_bits(kt);
  if (!bits) return VQS_ETYPE;
  pl->bits = bits;
  pl->ks = bits / 8;
  pl->mode = mode_of(kt, asc);
  pl->n = n;
  pl->nseg = nseg;
  pl->seed = o ? o->seed : 0;
  pl->rng_mode = VQS_HAS(o, rng_key) ? o->rng : (uint32_t)VQS_RNG_SFC64;
  if (pl->rng_mode > VQS_RNG_CHACHA20) return VQS_EINVAL;
  for (int i = 0; i < 8; i++) pl->rng_key[i] = pl->rng_mode ? o->rng_key[i] : 0u;
  pl->nb = (o && o->base_case) ? o->base_case : 256;
  if (pl->nb < 32 || pl->nb > 256) return VQS_EINVAL;
  const uint64_t lbk = local_buffer_keys(bits);
  pl->local = (o && o->local_keys) ? o->local_keys : (uint32_t)lbk;
  if (pl->local > lbk || pl->local < pl->nb) return VQS_EINVAL;
  // every LDS recursion level holds fewer than LOCAL_LIST_CAP ranges longer than nb
  if (pl->local / (pl->nb + 1) >= (uint32_t)LOCAL_LIST_CAP) {
    if (o && o->local_keys) return VQS_EINVAL;
    pl->local = (uint32_t)((LOCAL_LIST_CAP - 1) * (pl->nb + 1));
  }
  if (o && o->solo_max) {
    pl->solo = o->solo_max;
    if (pl->solo < pl->local) return VQS_EINVAL;
  } else {
    // ranges above 32K keys are partitioned by the device-wide level kernel, which
    // moves data faster than one workgroup's partitions (below that, a level's fixed
    // costs outweigh it: measured on 1e8 u64 and 2e8 u32; 48K: 1e8 u64 even, 1e8 Zipf
    // +2.5 %, 2.5e8 f32 -0.9 %); a few times more ranges than solo workgroups keep the
    // solo kernel busy on very large inputs, and on inputs too small to give it four
    // 32K-key ranges per workgroup the threshold drops towards the LDS capacity (2e7
    // u64: -3.4 %)
    uint64_t s = n / ((uint64_t)g.solo_grid * 16);
    const uint64_t floor_ = std::min<uint64_t>(1u << 15, n / ((uint64_t)g.solo_grid * 4));
    s = std::max<uint64_t>(s, std::max<uint64_t>(pl->local, floor_));
    s = std::min<uint64_t>(s, 1ull << 20);
    pl->solo = std::max<uint64_t>(s, pl->local);
  }
  // (level_mode is read only from a struct that holds it)
  const uint32_t lm = VQS_HAS(o, level_mode) ? o->level_mode : (uint32_t)VQS_LEVEL_AUTO;
  if (lm > VQS_LEVEL_RUNS) return VQS_EINVAL;
  // auto: runs for one array of 8- or 16-byte keys, whose top levels are a few long
  // ranges (long look-back chains); the look-back for narrower keys and for many
  // ranges at once (segments, learned buckets), where it measured faster
  pl->run_mode = lm == VQS_LEVEL_RUNS || (lm == VQS_LEVEL_AUTO && bits >= 64 && nseg == 1);
  pl->depth_limit = -1;
  uint32_t lim = depth_limit_for(std::max<uint64_t>(n, 2));
  if (o && o->depth_limit != 0) {
    pl->depth_limit = o->depth_limit > 0 ? o->depth_limit : 0;
    if (pl->depth_limit > 200) return VQS_EINVAL;
    lim = (uint32_t)pl->depth_limit;
  }
  pl->fb_limit = -1;
  uint32_t fb_lim = depth_limit_for(std::max<uint64_t>(n, 2));
  if (VQS_HAS(o, fallback_limit) && o->fallback_limit != 0) {
    pl->fb_limit = o->fallback_limit == VQS_FALLBACK_LIMIT_ZERO ? 0 : (int64_t)o->fallback_limit;
    if (pl->fb_limit > 200) return VQS_EINVAL;
    fb_lim = std::max<uint32_t>(fb_lim, (uint32_t)pl->fb_limit);
  }
  // A range reaches the paper's depth limit by level lim (one more when the ranges are
  // seeded at level 1); past it, fallback mode may take fb_lim more levels.
  // Levels 0 .. max_levels - 2 are launched.
  // (one more: in run mode a range leaving for the solo list is gathered by a copy
  // entry of the next level)
  pl->max_levels = (int)lim + (int)fb_lim + 5;
  pl->tile = VQS_HAS(o, tile_variant) ? (int)o->tile_variant : 0;
  if (pl->tile < 0 || pl->tile > 1) return VQS_EINVAL;
  const uint64_t T = level_tile_keys(bits, pl->tile);
  // a level holds at most n / (solo + 1) ranges longer than solo, and up to twice as
  // many copy entries
  pl->cap_lvl = 3 * (n / (pl->solo + 1)) + 4;
  pl->cap_tiles = n / T + 2 * pl->cap_lvl + 2;
  pl->inplace = VQS_HAS(o, inplace) ? (int)o->inplace : 0;
  pl->ip_steps = ip_steps_of(pl->ks);
  if (pl->inplace < 0 || pl->inplace > 1) return VQS_EINVAL;
  if (pl->inplace) {
    if (o->use_graph || o->method != VQS_METHOD_PLAIN) return VQS_EINVAL;
    // the solo kernel's in-place partitions keep their block tables in LDS
    if (o->solo_max && (o->solo_max < IP_SOLO_MIN || o->solo_max > IP_SOLO_MAX)) return VQS_EINVAL;
    pl->solo = std::min<uint64_t>(std::max<uint64_t>(pl->solo, IP_SOLO_MIN), IP_SOLO_MAX);
    pl->run_mode = 0;   // (level_mode and tile_variant do not apply)
    pl->tile = 0;
    pl->cap_lvl = n / (pl->solo + 1) + 4;
    pl->cap_tiles = n / ((uint64_t)IP_B * pl->ip_steps) + pl->cap_lvl + 2;
  }
  pl->cap_solo = nseg + 2ull * (uint64_t)pl->max_levels * pl->cap_lvl + n / FILL_CHUNK + 64;
  return VQS_OK;
}

size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

// Capacities a workspace is carved for.
struct Caps {
  uint64_t scratch_bytes, lvl, tiles, solo;
  int levels;
  uint64_t ip_stash_bytes, ip_pfx;   // in-place levels: saved keys, block prefix entries
};

Caps caps_of(const Plan& pl) {
  if (pl.inplace)
    return Caps{0, pl.cap_lvl, pl.cap_tiles, pl.cap_solo, pl.max_levels,
                pl.cap_lvl * IP_STASH * (uint64_t)pl.ks, pl.cap_tiles * pl.ip_steps};
  return Caps{(pl.n + 32) * (uint64_t)pl.ks + 64, pl.cap_lvl, pl.cap_tiles, pl.cap_solo, pl.max_levels, 0, 0};
}

// Layout of a workspace with capacities c: returns its size in bytes and, when mem is
// not null, points p's buffers into mem (which must be 256-byte aligned).
size_t carve(char* mem, const Caps& c, Params* p) {
  size_t off = 0;
  auto take = [&](size_t b) {
    size_t o = off;
    off = align_up(off + b, 256);
    return o;
  };
  const size_t o_scratch = take(c.scratch_bytes);
  const size_t o_seg0 = take(c.lvl * sizeof(Seg));
  const size_t o_seg1 = take(c.lvl * sizeof(Seg));
  const size_t o_tb0 = take(c.lvl * 8);
  const size_t o_tb1 = take(c.lvl * 8);
  const size_t o_ctr = take((size_t)c.levels * sizeof(LevelCtr));
  const size_t o_flags = take(c.tiles * 8);
  const size_t o_tmin = take(c.tiles * sizeof(u128k));
  const size_t o_trmin = take(c.tiles * sizeof(u128k));
  const size_t o_run0 = take(c.tiles * sizeof(TileRun));
  const size_t o_run1 = take(c.tiles * sizeof(TileRun));
  const size_t o_tref = take(c.tiles * sizeof(TileRef));
  const size_t o_tnl = take(c.tiles * sizeof(uint32_t));
  const size_t o_solo = take(c.solo * sizeof(Seg));
  const size_t o_sctr = take(sizeof(SoloCtr));
  const size_t o_sord = take(c.solo * 4);
  const size_t o_stats = take(sizeof(DevStats));
  const size_t o_err = take(16);
  const size_t o_ipst = take(c.ip_stash_bytes);
  const size_t o_ippf = take(c.ip_pfx * 8);
  const size_t o_iprg = take(c.ip_stash_bytes ? c.lvl * sizeof(IpRange) : 0);
  if (!mem) return off;
  p->ip_stash = mem + o_ipst;
  p->ip_pfx = (unsigned long long*)(mem + o_ippf);
  p->ip_rng = (IpRange*)(mem + o_iprg);
  // the tile ranges share run mode's per-tile left counts (run mode is off in place)
  p->ip_tseg = (uint32_t*)(mem + o_tnl);
  p->scratch = mem + o_scratch;  // re-based per call to the keys' alignment
  p->lvl_segs[0] = (Seg*)(mem + o_seg0);
  p->lvl_segs[1] = (Seg*)(mem + o_seg1);
  p->lvl_tbase[0] = (unsigned long long*)(mem + o_tb0);
  p->lvl_tbase[1] = (unsigned long long*)(mem + o_tb1);
  p->lvl_ctr = (LevelCtr*)(mem + o_ctr);
  p->flags = (unsigned long long*)(mem + o_flags);
  p->tilemin = (u128k*)(mem + o_tmin);
  p->tilermin = (u128k*)(mem + o_trmin);
  p->runs[0] = (TileRun*)(mem + o_run0);
  p->runs[1] = (TileRun*)(mem + o_run1);
  p->tref = (TileRef*)(mem + o_tref);
  p->tnl = (uint32_t*)(mem + o_tnl);
  p->solo = (Seg*)(mem + o_solo);
  p->solo_ctr = (SoloCtr*)(mem + o_sctr);
  p->solo_order = (uint32_t*)(mem + o_sord);
  p->stats = (DevStats*)(mem + o_stats);
  p->err = (unsigned int*)(mem + o_err);
  p->cap_lvl = c.lvl;
  p->cap_tiles = c.tiles;
  p->cap_solo = c.solo;
  return off;
}

void set_caps(Workspace* ws, const Caps& c) {
  ws->cap_scratch_bytes = c.scratch_bytes;
  ws->cap_lvl = c.lvl;
  ws->cap_tiles = c.tiles;
  ws->cap_solo = c.solo;
  ws->cap_levels = c.levels;
  ws->cap_ip_stash = c.ip_stash_bytes;
  ws->cap_ip_pfx = c.ip_pfx;
}

Caps caps_held(const Workspace* ws) {
  return Caps{ws->cap_scratch_bytes, ws->cap_lvl, ws->cap_tiles, ws->cap_solo, ws->cap_levels, ws->cap_ip_stash,
              ws->cap_ip_pfx};
}

// Allocate (or reuse) the workspace for a plan.  Caller holds g_mu.
int ensure_workspace(Workspace* ws, const Plan& pl) {
  const Caps need = caps_of(pl);
  if (ws->mem && need.scratch_bytes <= ws->cap_scratch_bytes && need.lvl <= ws->cap_lvl &&
      need.tiles <= ws->cap_tiles && need.solo <= ws->cap_solo && need.levels <= ws->cap_levels &&
      need.ip_stash_bytes <= ws->cap_ip_stash && need.ip_pfx <= ws->cap_ip_pfx) {
    if (ws->p_external) {   // the last call used a caller's workspace
      const Caps c = caps_held(ws);
      carve(ws->mem, c, &ws->p);
      ws->p_levels = c.levels;
      ws->p_external = false;
    }
    return VQS_OK;
  }
  if (ws->mem) {
    (void)hipStreamSynchronize(ws->stream);
    if (ws->graph) {
      (void)hipGraphExecDestroy(ws->graph);
      ws->graph = nullptr;
      ws->graph_valid = false;
    }
    (void)hipFree(ws->mem);
    ws->mem = nullptr;
  }
  const Caps c{std::max(need.scratch_bytes, ws->cap_scratch_bytes), std::max(need.lvl, ws->cap_lvl),
               std::max(need.tiles, ws->cap_tiles), std::max(need.solo, ws->cap_solo),
               std::max(need.levels, ws->cap_levels), std::max(need.ip_stash_bytes, ws->cap_ip_stash),
               std::max(need.ip_pfx, ws->cap_ip_pfx)};
  const size_t bytes = carve(nullptr, c, nullptr);
  void* mem = nullptr;
  if (hipMalloc(&mem, bytes) != hipSuccess || !mem) {
    (void)hipGetLastError();
    return VQS_ENOMEM;
  }
  ws->mem = (char*)mem;
  ws->bytes = bytes;
  set_caps(ws, c);
  carve(ws->mem, c, &ws->p);
  ws->p_levels = c.levels;
  ws->p_external = false;
  if (!ws->host_pinned && hipHostMalloc((void**)&ws->host_pinned, 4096, hipHostMallocDefault) != hipSuccess) {
    ws->host_pinned = nullptr;
    return VQS_ENOMEM;
  }
  if (hipMemsetAsync(ws->p.stats, 0, sizeof(DevStats), ws->stream) != hipSuccess) return VQS_EHIP;
  return VQS_OK;
}

Workspace* workspace_for(hipStream_t s) {
  int dev = 0;
  (void)hipGetDevice(&dev);
  auto key = std::make_pair(dev, s);
  auto it = g_ws.find(key);
  if (it != g_ws.end()) return it->second.get();
  auto ws = std::make_unique<Workspace>();
  ws->device = dev;
  ws->stream = s;
  Workspace* r = ws.get();
  g_ws[key] = std::move(ws);
  return r;
}

// Levels launched before the host reads whether work is left: a read stalls the GPU
// for a round trip (about 35 us), a level launched without work costs two launches
// that return at once (a few us).  First batch: log2(n / solo threshold), the
// halvings a range takes to reach the solo list, plus room for uneven pivots;
// afterwards LEVEL_BATCH_NEXT at a time.
constexpr int LEVEL_BATCH_NEXT = 4;
int level_batch(const Plan& pl) {
  int batch = 6;
  for (uint64_t x = pl.n / std::max<uint64_t>(pl.solo, 1); x > 1; x >>= 1) batch++;
  return batch;
}

template <int B, int LI>
hipError_t launch_all(Workspace* ws, const Params& base, const Plan& pl, const Geometry& g,
                      const int64_t* offsets, uint64_t nseg, bool capture, int* levels_out) {
  hipStream_t s = ws->stream;
  hipError_t e = ws->timed(0, -1, [&] { return Launch<B>::clear(base, s); });
  if (e != hipSuccess) return e;
  e = ws->timed(1, -1, [&] { return LaunchLevel<B, LI>::seed(base, offsets, nseg, s); });
  if (e != hipSuccess) return e;
  // the level loop: launch levels in batches, then read the next level's counter
  int L = base.seed_level;
  if (pl.n > pl.solo && base.run_mode) {
    // run mode: plan(L) plans level L-1's ranges into level L and gives level L its
    // pivots, then level(L) partitions it; after the last level with work, one more
    // plan routes its children
    auto step = [&](int lv, bool part) -> hipError_t {
      Params p = base;
      p.level = lv;
      hipError_t e2 = ws->timed(8, lv, [&] { return LaunchLevel<B, LI>::plan(p, g.plan_grid, s); });
      if (e2 != hipSuccess || !part) return e2;
      return ws->timed(2, lv, [&] { return LaunchLevel<B, LI>::level(p, g.level_grid, s); });
    };
    if (capture) {
      for (; L < pl.max_levels - 1; L++) {
        e = step(L, true);
        if (e != hipSuccess) return e;
      }
      e = step(L, false);
      if (e != hipSuccess) return e;
    } else {
      int batch = level_batch(pl);
      for (;;) {
        const int upto = std::min(L + batch, pl.max_levels - 1);
        for (; L < upto; L++) {
          e = step(L, true);
          if (e != hipSuccess) return e;
        }
        // the last launched level had no work: nothing is left to plan
        e = hipMemcpyAsync(ws->ctr_word(), &base.lvl_ctr[L - 1].packed, 8, hipMemcpyDeviceToHost, s);
        if (e != hipSuccess) return e;
        e = hipStreamSynchronize(s);
        if (e != hipSuccess) return e;
        if (ws->ctr_word()[0] == 0) break;
        if (L >= pl.max_levels - 1) {
          e = step(L, false);
          if (e != hipSuccess) return e;
          break;
        }
        batch = LEVEL_BATCH_NEXT;
      }
    }
  } else if (pl.n > pl.solo && base.inplace) {
    // in place: pivots, then the counting and partition launches, per level
    int batch = capture ? pl.max_levels : level_batch(pl);
    for (;;) {
      const int upto = std::min(L + batch, pl.max_levels - 1);
      for (; L < upto; L++) {
        Params p = base;
        p.level = L;
        e = ws->timed(8, L, [&] { return LaunchLevel<B, LI>::pivots(p, g.pivot_grid, s); });
        if (e != hipSuccess) return e;
        e = ws->timed(2, L, [&] { return Launch<B>::ip_level(p, g.level_grid, s); });
        if (e != hipSuccess) return e;
      }
      if (L >= pl.max_levels - 1 || capture) break;
      e = hipMemcpyAsync(ws->ctr_word(), &base.lvl_ctr[L].packed, 8, hipMemcpyDeviceToHost, s);
      if (e != hipSuccess) return e;
      e = hipStreamSynchronize(s);
      if (e != hipSuccess) return e;
      if (ws->ctr_word()[0] == 0) break;
      batch = LEVEL_BATCH_NEXT;
    }
  } else if (pl.n > pl.solo) {
    if (capture) {
      for (; L < pl.max_levels - 1; L++) {
        Params p = base;
        p.level = L;
        e = ws->timed(8, L, [&] { return LaunchLevel<B, LI>::pivots(p, g.pivot_grid, s); });
        if (e != hipSuccess) return e;
        e = ws->timed(2, L, [&] { return LaunchLevel<B, LI>::level(p, g.level_grid, s); });
        if (e != hipSuccess) return e;
      }
    } else {
      int batch = level_batch(pl);
      for (;;) {
        const int upto = std::min(L + batch, pl.max_levels - 1);
        for (; L < upto; L++) {
          Params p = base;
          p.level = L;
          e = ws->timed(8, L, [&] { return LaunchLevel<B, LI>::pivots(p, g.pivot_grid, s); });
          if (e != hipSuccess) return e;
          e = ws->timed(2, L, [&] { return LaunchLevel<B, LI>::level(p, g.level_grid, s); });
          if (e != hipSuccess) return e;
        }
        if (L >= pl.max_levels - 1) break;
        e = hipMemcpyAsync(ws->ctr_word(), &base.lvl_ctr[L].packed, 8, hipMemcpyDeviceToHost, s);
        if (e != hipSuccess) return e;
        e = hipStreamSynchronize(s);
        if (e != hipSuccess) return e;
        if (ws->ctr_word()[0] == 0) break;
        batch = LEVEL_BATCH_NEXT;
      }
    }
  }
  *levels_out = L;
  return ws->timed(3, -1, [&] { return Launch<B>::solo(base, g.solo_grid, s); });
}

hipError_t dispatch_launch(Workspace* ws, const Params& base, const Plan& pl, const Geometry& g,
                           const int64_t* offsets, uint64_t nseg, bool capture, int* levels) {
#define VQS_LAUNCH_ALL(B)                                                                              \
  return pl.tile ? launch_all<B, level_chunks_half(B)>(ws, base, pl, g, offsets, nseg, capture, levels) \
                 : launch_all<B, level_chunks(B)>(ws, base, pl, g, offsets, nseg, capture, levels)
  switch (pl.bits) {
    case 16: VQS_LAUNCH_ALL(16);
    case 32: VQS_LAUNCH_ALL(32);
    case 64: VQS_LAUNCH_ALL(64);
    default: VQS_LAUNCH_ALL(128);
  }
#undef VQS_LAUNCH_ALL
}

int check_offsets_host(const int64_t* offsets, uint64_t nseg, uint64_t* total, hipStream_t s) {
  int64_t* h = (int64_t*)malloc((nseg + 1) * sizeof(int64_t));
  if (!h) return VQS_ENOMEM;
  if (hipMemcpyAsync(h, offsets, (nseg + 1) * sizeof(int64_t), hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess) {
    free(h);
    return VQS_EHIP;
  }
  int rc = VQS_OK;
  if (h[0] < 0) rc = VQS_EOFFSETS;
  for (uint64_t i = 0; i < nseg && rc == VQS_OK; i++)
    if (h[i + 1] < h[i]) rc = VQS_EOFFSETS;
  *total = rc == VQS_OK ? (uint64_t)h[nseg] : 0;
  free(h);
  return rc;
}

int learned_locked(Workspace* ws, void* keys, uint64_t n, const vqs_options* o, hipStream_t stream, bool fit_only,
                   float* params_out);

// Per-call parameters for keys from a carved workspace's buffers.
void init_params(Params* base, const Params& carved, void* keys, uint64_t n, const Plan& pl) {
  const uintptr_t addr = (uintptr_t)keys;
  Params& b = *base;
  b = carved;
  b.keys = keys;
  b.off = (int)((addr % 16) / (uintptr_t)pl.ks);
  // scratch shares the keys' offset from a 16-byte boundary
  b.scratch = (void*)(((uintptr_t)carved.scratch + 15) / 16 * 16 + (addr % 16));
  b.n_total = n;
  b.mode = pl.mode;
  b.seed = pl.seed;
  b.rng_mode = pl.rng_mode;
  for (int i = 0; i < 8; i++) b.rng_key[i] = pl.rng_key[i];
  b.nb = pl.nb;
  b.local_cap = pl.local;
  b.solo_max = pl.solo;
  b.max_levels = pl.max_levels;
  b.level = 0;
  b.seed_level = 0;
  b.fixed_limit = pl.depth_limit;
  b.fb_limit = pl.fb_limit;
  b.run_mode = pl.run_mode;
  b.inplace = pl.inplace;
  b.ip_steps = pl.ip_steps;
}

// Prepare base parameters for keys on ws (caller holds g_mu).
int prepare(Workspace* ws, void* keys, uint64_t n, uint64_t nseg, int kt, int asc, const vqs_options* o, Plan* pl,
            Params* base) {
  const Geometry g = geometry(ws->device);
  int rc = make_plan(n, nseg, kt, asc, o, g, pl);
  if (rc != VQS_OK) return rc;
  if (VQS_HAS(o, workspace_bytes) && o->workspace) {
    // the caller's workspace: carved for this call, nothing allocated
    const Caps c = caps_of(*pl);
    if (carve(nullptr, c, nullptr) > o->workspace_bytes) return VQS_ESIZE;
    carve((char*)o->workspace, c, &ws->p);
    ws->p_levels = c.levels;
    ws->p_external = true;
  } else {
    rc = ensure_workspace(ws, *pl);
    if (rc != VQS_OK) return rc;
  }
  init_params(base, ws->p, keys, n, *pl);
  return VQS_OK;
}

// The plain method on keys (one array, or nseg segments); caller holds g_mu.
int sort_locked(Workspace* ws, void* keys, const int64_t* offsets, uint64_t nseg, uint64_t n, int kt, int asc,
                const vqs_options* o, hipStream_t stream) {
  Plan pl;
  Params base;
  int rc = prepare(ws, keys, n, nseg, kt, asc, o, &pl, &base);
  if (rc != VQS_OK) return rc;
  const Geometry g = geometry(ws->device);
  ws->have_result = false;
  ws->learned_ran = false;
  int levels = 0;
  hipError_t e;
  const bool use_graph = o && o->use_graph && offsets;
  if (use_graph) {
    GraphKey gk{base.stats, keys, offsets, nseg, n, kt, asc, pl.seed, pl.depth_limit, pl.fb_limit, pl.nb, pl.local,
                pl.solo, pl.run_mode, pl.tile, pl.rng_mode, {}, pl.inplace};
    for (int i = 0; i < 8; i++) gk.rng_key[i] = pl.rng_key[i];
    if (!(ws->graph_valid && !(gk < ws->graph_key) && !(ws->graph_key < gk))) {
      if (ws->graph) {
        (void)hipGraphExecDestroy(ws->graph);
        ws->graph = nullptr;
      }
      ws->graph_valid = false;
      hipStream_t cap;
      if (hipStreamCreateWithFlags(&cap, hipStreamNonBlocking) != hipSuccess) return VQS_EHIP;
      hipStream_t saved = ws->stream;
      ws->stream = cap;
      ws->capturing = true;
      e = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal);
      if (e == hipSuccess) e = dispatch_launch(ws, base, pl, g, offsets, nseg, true, &levels);
      hipGraph_t graph = nullptr;
      hipError_t e2 = hipStreamEndCapture(cap, &graph);
      ws->stream = saved;
      ws->capturing = false;
      if (e == hipSuccess) e = e2;
      if (e == hipSuccess) e = hipGraphInstantiate(&ws->graph, graph, nullptr, nullptr, 0);
      if (graph) (void)hipGraphDestroy(graph);
      (void)hipStreamDestroy(cap);
      if (e != hipSuccess) return VQS_EHIP;
      ws->graph_key = gk;
      ws->graph_valid = true;
    }
    e = hipGraphLaunch(ws->graph, stream);
    if (e != hipSuccess) return VQS_EHIP;
    ws->last_levels = pl.max_levels - 1;
    ws->have_result = true;
    ws->seq = ++g_seq;
    return VQS_OK;
  }
  e = dispatch_launch(ws, base, pl, g, offsets, nseg, false, &levels);
  if (e != hipSuccess) return VQS_EHIP;
  ws->last_levels = levels;
  ws->have_result = true;
  ws->seq = ++g_seq;
  return VQS_OK;
}

int sort_impl(void* keys, const int64_t* offsets, uint64_t nseg, uint64_t n, int kt, int asc,
              const vqs_options* o, hipStream_t stream) {
  if (o && o->struct_size != 0 && o->struct_size < offsetof(vqs_options, train_steps)) return VQS_EINVAL;
  const int bits = key_bits(kt);
  if (!bits) return VQS_ETYPE;
  if (asc != 0 && asc != 1) return VQS_EINVAL;
  if (o && o->method > VQS_METHOD_LEARNED) return VQS_EINVAL;
  const bool learned = o && o->method == VQS_METHOD_LEARNED;
  if (learned && (kt != VQS_U64 || offsets || !asc)) return VQS_EINVAL;
  if (learned && VQS_HAS(o, inplace) && o->inplace) return VQS_EINVAL;   // its buckets need the scratch
  if (VQS_HAS(o, workspace_bytes) && o->workspace && (learned || (uintptr_t)o->workspace % 256)) return VQS_EINVAL;
  if (n == 0) return VQS_OK;
  if (!keys) return VQS_EINVAL;
  const int ks = bits / 8;
  if ((uintptr_t)keys % (uintptr_t)std::min(ks, 16)) return VQS_EINVAL;
  std::lock_guard<std::mutex> lock(g_mu);
  Workspace* ws = workspace_for(stream);
  if (learned) return learned_locked(ws, keys, n, o, stream, false, nullptr);
  return sort_locked(ws, keys, offsets, nseg, n, kt, asc, o, stream);
}

// ---- learned splitter ------------------------------------------------------------------

int ensure_learned(Workspace* ws, uint64_t m, uint64_t nchunks) {
  if (ws->lmem && m <= ws->lcap_m && nchunks <= ws->lcap_chunks) return VQS_OK;
  if (ws->lmem) {
    (void)hipStreamSynchronize(ws->stream);
    (void)hipFree(ws->lmem);
    ws->lmem = nullptr;
  }
  m = std::max(m, ws->lcap_m);
  nchunks = std::max(nchunks, ws->lcap_chunks);
  size_t off = 0;
  auto take = [&](size_t b) {
    size_t o = off;
    off = align_up(off + b, 256);
    return o;
  };
  const size_t o_sample = take(m * 8), o_x = take(m * 4), o_t = take(m * 4), o_p = take(MLP_NBLOCK * 4),
               o_mom = take((2 * MLP_NPARAM + 1) * 4), o_thr = take(NBUCKET * 8), o_nv = take(16),
               o_hist = take(nchunks * NBUCKET * 4), o_tot = take(NBUCKET * 8), o_off = take((NBUCKET + 1) * 8),
               o_sum = take(64);
  void* mem = nullptr;
  if (hipMalloc(&mem, off) != hipSuccess || !mem) {
    (void)hipGetLastError();
    return VQS_ENOMEM;
  }
  char* b = (char*)mem;
  ws->lmem = b;
  ws->lcap_m = m;
  ws->lcap_chunks = nchunks;
  ws->l_sample = (uint64_t*)(b + o_sample);
  ws->l_x = (float*)(b + o_x);
  ws->l_t = (float*)(b + o_t);
  ws->l_params = (float*)(b + o_p);
  ws->l_moments = (float*)(b + o_mom);
  ws->l_thr = (uint64_t*)(b + o_thr);
  ws->l_nvalid = (uint32_t*)(b + o_nv);
  ws->l_hist = (uint32_t*)(b + o_hist);
  ws->l_totals = (uint64_t*)(b + o_tot);
  ws->l_offsets = (int64_t*)(b + o_off);
  ws->l_summary = (uint64_t*)(b + o_sum);
  return VQS_OK;
}

Workspace* inner_for(Workspace* ws) {
  if (!ws->inner) {
    ws->inner = std::make_unique<Workspace>();
    ws->inner->device = ws->device;
    ws->inner->stream = ws->stream;
  }
  return ws->inner.get();
}

// Sample, sort the sample, targets, model init and training; then (unless fit_only)
// thresholds, histogram, scan, scatter into scratch and the plain method on the 256
// buckets.  Caller holds g_mu.
int learned_locked(Workspace* ws, void* keys, uint64_t n, const vqs_options* o, hipStream_t stream, bool fit_only,
                   float* params_out) {
  const float frac = (o && o->sample_fraction > 0.f) ? o->sample_fraction : 0.01f;
  const uint32_t steps = (o && o->train_steps) ? o->train_steps : 100;
  const uint32_t batch = (o && o->batch) ? std::min<uint32_t>(o->batch, MLP_MAX_BATCH) : MLP_MAX_BATCH;
  const float lr = (o && o->learning_rate > 0.f) ? o->learning_rate : 0.003f;
  const float over = (o && o->overflow_factor > 0.f) ? o->overflow_factor : 2.0f;
  const uint64_t model_seed = (o && o->model_seed) ? o->model_seed : 16;
  const uint64_t sample_seed = (o && o->sample_seed) ? o->sample_seed : 17;
  if (n < 64) return fit_only ? VQS_EINVAL : sort_locked(ws, keys, nullptr, 1, n, VQS_U64, 1, o, stream);
  uint64_t chunks = (uint64_t)((double)frac * (double)n / 8.0);
  chunks = std::max<uint64_t>(chunks, 8);
  chunks = std::min<uint64_t>(chunks, n / 8);
  const uint64_t m = chunks * 8;
  const uint64_t nchunks = (n + (uint64_t)LEARN_TILE * CHUNK_TILES - 1) / ((uint64_t)LEARN_TILE * CHUNK_TILES);
  // the workspace for the final plain phase first: it owns the scatter target
  Plan pl;
  Params base;
  vqs_options plain{};
  if (o) plain = *o;
  plain.struct_size = sizeof(vqs_options);
  plain.method = VQS_METHOD_PLAIN;
  int rc = VQS_OK;
  if (!fit_only) {
    rc = prepare(ws, keys, n, NBUCKET, VQS_U64, 1, &plain, &pl, &base);
    if (rc != VQS_OK) return rc;
  }
  rc = ensure_learned(ws, m, nchunks);
  if (rc != VQS_OK) return rc;
  ws->have_result = false;
  ws->learned_ran = false;
  hipError_t e = ws->timed(4, -1, [&] { return launch_sample((const uint64_t*)keys, n, ws->l_sample, chunks, sample_seed, stream); });
  if (e != hipSuccess) return VQS_EHIP;
  Workspace* in = inner_for(ws);
  in->stream = stream;
  vqs_options sopt{};
  sopt.struct_size = sizeof(vqs_options);
  sopt.seed = o ? o->seed : 0;
  // (the sample is small: the solo threshold rule gives its sort solo ranges of the
  // LDS capacity, which keep the solo kernel's workgroups busy)
  rc = sort_locked(in, ws->l_sample, nullptr, 1, m, VQS_U64, 1, &sopt, stream);
  if (rc != VQS_OK) return rc;
  e = ws->timed(5, -1, [&] {
    hipError_t r = launch_targets(ws->l_sample, m, ws->l_x, ws->l_t, stream);
    if (r == hipSuccess) r = launch_init(ws->l_params, model_seed, ws->l_x, m, stream);
    if (r == hipSuccess) r = hipMemsetAsync(ws->l_moments, 0, (2 * MLP_NPARAM + 1) * 4, stream);
    if (r == hipSuccess && steps > 0) {
      TrainArgs a{ws->l_x, ws->l_t, m, steps, batch, lr, sample_seed, 0};
      r = launch_train(ws->l_params, ws->l_moments, a, stream);
    }
    return r;
  });
  if (e != hipSuccess) return VQS_EHIP;
  if (fit_only) {
    if (params_out &&
        hipMemcpyAsync(params_out, ws->l_params, MLP_NBLOCK * 4, hipMemcpyDeviceToDevice, stream) != hipSuccess)
      return VQS_EHIP;
    return VQS_OK;
  }
  e = ws->timed(6, -1, [&] { return launch_thresholds(ws->l_params, ws->l_thr, ws->l_nvalid, stream); });
  if (e != hipSuccess) return VQS_EHIP;
  e = ws->timed(7, -1, [&] {
    hipError_t r = launch_histogram((const uint64_t*)keys, n, ws->l_thr, ws->l_nvalid, ws->l_hist, nchunks, stream);
    if (r == hipSuccess) r = launch_scan(ws->l_hist, nchunks, ws->l_totals, stream);
    if (r == hipSuccess) r = launch_offsets(ws->l_totals, n, over, ws->l_offsets, ws->l_summary, stream);
    if (r == hipSuccess)
      r = launch_scatter((const uint64_t*)keys, n, ws->l_thr, ws->l_nvalid, ws->l_hist, nchunks, ws->l_offsets,
                         (uint64_t*)base.scratch, stream);
    return r;
  });
  if (e != hipSuccess) return VQS_EHIP;
  // the 256 buckets, now in scratch, are sorted as segments starting at level 1
  base.seed_level = 1;
  int levels = 0;
  const Geometry g = geometry(ws->device);
  e = dispatch_launch(ws, base, pl, g, ws->l_offsets, NBUCKET, false, &levels);
  if (e != hipSuccess) return VQS_EHIP;
  ws->last_levels = levels;
  ws->have_result = true;
  ws->seq = ++g_seq;
  ws->learned_ran = true;
  return VQS_OK;
}

// ---- stable sort ---------------------------------------------------------------------------

int stable_sort(void* keys, uint64_t n, int kt, int asc, uint64_t* rows, const vqs_options* o, hipStream_t stream) {
  if (o && o->struct_size != 0 && o->struct_size < offsetof(vqs_options, train_steps)) return VQS_EINVAL;
  const int bits = key_bits(kt);
  if (!bits || bits > 64) return VQS_ETYPE;
  if (asc != 0 && asc != 1) return VQS_EINVAL;
  if (o && o->method != VQS_METHOD_PLAIN) return VQS_EINVAL;
  if (VQS_HAS(o, workspace_bytes) && o->workspace) return VQS_EINVAL;
  if (n == 0) return VQS_OK;
  if (!keys) return VQS_EINVAL;
  if ((uintptr_t)keys % (uintptr_t)(bits / 8) || (rows && (uintptr_t)rows % 8)) return VQS_EINVAL;
  // (key << 32 | row) fits a u64 for keys of up to 32 bits and rows below 2^32
  const int comp = (bits <= 32 && n <= (1ull << 32)) ? COMP64 : COMP128;
  const size_t cbytes = (size_t)n * (comp == COMP64 ? 8 : 16);
  std::lock_guard<std::mutex> lock(g_mu);
  Workspace* ws = workspace_for(stream);
  if (cbytes > ws->scap) {
    if (ws->smem) {
      (void)hipStreamSynchronize(ws->stream);
      (void)hipFree(ws->smem);
      ws->smem = nullptr;
      ws->scap = 0;
    }
    void* m = nullptr;
    if (hipMalloc(&m, cbytes) != hipSuccess || !m) {
      (void)hipGetLastError();
      return VQS_ENOMEM;
    }
    ws->smem = (char*)m;
    ws->scap = cbytes;
  }
  ws->stream = stream;
  const int mode = mode_of(kt, asc);
  if (launch_stable_pack(keys, n, bits, mode, comp, ws->smem, stream) != hipSuccess) return VQS_EHIP;
  vqs_options plain{};
  if (o) std::memcpy(&plain, o, std::min<size_t>(o->struct_size ? o->struct_size : sizeof(vqs_options),
                                                sizeof(vqs_options)));
  plain.struct_size = sizeof(vqs_options);
  plain.method = VQS_METHOD_PLAIN;
  plain.use_graph = 0;
  plain.workspace = nullptr;
  plain.workspace_bytes = 0;
  const int rc = sort_locked(ws, ws->smem, nullptr, 1, n, comp == COMP64 ? VQS_U64 : VQS_U128, 1, &plain, stream);
  if (rc != VQS_OK) return rc;
  if (launch_stable_unpack(ws->smem, n, bits, mode, comp, keys, rows, stream) != hipSuccess) return VQS_EHIP;
  return VQS_OK;
}

// ---- allocation-free entry point -------------------------------------------------------

constexpr int NOALLOC_MAX_DEVICES = 64;

// Per-device state of vqs_sort_noalloc.  Nothing here owns memory: ws carves its
// buffers from the device's copy of `scratch` and reads the level counter into its
// pageable host word.
struct NoAlloc {
  bool ready = false;
  char* ptr = nullptr;                   // this device's copy of `scratch`
  Geometry geom{};
  Workspace ws;   // no pinned host word: level counters are read into ws.host_word
};

NoAlloc g_noalloc[NOALLOC_MAX_DEVICES];

int current_device() {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) {
    (void)hipGetLastError();
    dev = 0;
  }
  return dev;
}

// The workspace holding the newest result of a call on (current device, s).
Workspace* latest_ws(hipStream_t s) {
  const int dev = current_device();
  Workspace* best = nullptr;
  auto it = g_ws.find(std::make_pair(dev, s));
  if (it != g_ws.end()) best = it->second.get();
  if (dev >= 0 && dev < NOALLOC_MAX_DEVICES) {
    Workspace* na = &g_noalloc[dev].ws;
    if (na->have_result && na->stream == s && (!best || na->seq > best->seq)) best = na;
  }
  return best;
}

// First call on device dev (current): the device address of its copy of `scratch`.
// Caller holds g_mu.
int noalloc_setup(int dev) {
  NoAlloc& na = g_noalloc[dev];
  if (na.ready) return VQS_OK;
  void* ptr = nullptr;
  const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !ptr) {
    (void)hipGetLastError();
    return VQS_EHIP;
  }
  na.ptr = (char*)ptr;
  na.geom = geometry_of(dev);
  na.ws.owned = false;
  na.ws.no_profile = true;
  na.ws.device = dev;
  na.ws.mem = na.ptr;
  na.ready = true;
  return VQS_OK;
}

int noalloc_sort(void* keys, uint64_t n, int kt, int asc, const vqs_options* o, hipStream_t stream) {
  if (o && o->struct_size != 0 && o->struct_size < offsetof(vqs_options, train_steps)) return VQS_EINVAL;
  const int bits = key_bits(kt);
  if (!bits) return VQS_ETYPE;
  if (asc != 0 && asc != 1) return VQS_EINVAL;
  if (o && (o->method != VQS_METHOD_PLAIN || o->use_graph)) return VQS_EINVAL;
  if (VQS_HAS(o, workspace_bytes) && o->workspace) return VQS_EINVAL;
  if (n == 0) return VQS_OK;
  if (!keys) return VQS_EINVAL;
  if ((uintptr_t)keys % (uintptr_t)std::min(bits / 8, 16)) return VQS_EINVAL;
  std::lock_guard<std::mutex> lock(g_mu);
  const int dev = current_device();
  if (dev < 0 || dev >= NOALLOC_MAX_DEVICES) return VQS_EINVAL;
  int rc = noalloc_setup(dev);
  if (rc != VQS_OK) return rc;
  NoAlloc& na = g_noalloc[dev];
  Plan pl;
  rc = make_plan(n, 1, kt, asc, o, na.geom, &pl);
  if (rc != VQS_OK) return rc;
  const Caps c = caps_of(pl);
  if (carve(nullptr, c, nullptr) > (size_t)VQS_NOALLOC_SCRATCH_BYTES) return VQS_ESIZE;
  Workspace* ws = &na.ws;
  ws->stream = stream;
  ws->have_result = false;
  ws->learned_ran = false;
  ws->bytes = (size_t)VQS_NOALLOC_SCRATCH_BYTES;
  set_caps(ws, c);
  carve(ws->mem, c, &ws->p);
  ws->p_levels = c.levels;
  Params base;
  init_params(&base, ws->p, keys, n, pl);
  int levels = 0;
  // clear_kernel zeroes every counter, flag and statistic the call reads
  if (dispatch_launch(ws, base, pl, na.geom, nullptr, 1, false, &levels) != hipSuccess) return VQS_EHIP;
  ws->last_levels = levels;
  ws->have_result = true;
  ws->seq = ++g_seq;
  return VQS_OK;
}

}  // namespace

}  // namespace vqs

using namespace vqs;

extern "C" {

int vqs_sort_ex(void* keys, uint64_t n, int key_type, int ascending, const vqs_options* options, void* stream) {
  return sort_impl(keys, nullptr, 1, n, key_type, ascending, options, (hipStream_t)stream);
}

int vqs_sort(void* keys, uint64_t n, int key_type, int ascending) {
  return vqs_sort_ex(keys, n, key_type, ascending, nullptr, nullptr);
}

int vqs_sort_noalloc(void* keys, uint64_t n, int key_type, int ascending, const vqs_options* options,
                     void* stream) {
  return noalloc_sort(keys, n, key_type, ascending, options, (hipStream_t)stream);
}

int vqs_sort_stable(void* keys, uint64_t n, int key_type, int ascending, uint64_t* rows,
                    const vqs_options* options, void* stream) {
  return stable_sort(keys, n, key_type, ascending, rows, options, (hipStream_t)stream);
}

int vqs_sort_segmented_ex(void* keys, const int64_t* offsets, uint64_t nseg, int key_type, int ascending,
                          const vqs_options* options, void* stream) {
  if (!key_bits(key_type)) return VQS_ETYPE;
  if (nseg == 0) return VQS_OK;
  if (!offsets) return VQS_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  if (options && options->struct_size != 0 && options->struct_size < offsetof(vqs_options, train_steps))
    return VQS_EINVAL;
  // total key count = offsets[nseg] (and the scratch size): given by the caller, or
  // read once
  const uint64_t given = VQS_HAS(options, total_keys) ? options->total_keys : 0;
  uint64_t total = 0;
  if (options && options->validate) {
    int rc = check_offsets_host(offsets, nseg, &total, s);
    if (rc != VQS_OK) return rc;
    if (given && given != total) return VQS_EOFFSETS;
  } else if (given) {
    total = given;
  } else {
    int64_t last = 0;
    if (hipMemcpyAsync(&last, offsets + nseg, sizeof(int64_t), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
      return VQS_EHIP;
    if (last < 0) return VQS_EOFFSETS;
    total = (uint64_t)last;
  }
  return sort_impl(keys, offsets, nseg, total, key_type, ascending, options, s);
}

int vqs_autotune_segmented(const void* keys, const int64_t* offsets, uint64_t nseg, int key_type, int ascending,
                           uint64_t max_keys, vqs_options* options, float* best_ms, void* stream) {
  const int bits = key_bits(key_type);
  if (!bits) return VQS_ETYPE;
  if (!keys || !offsets || !options || nseg == 0 || (ascending != 0 && ascending != 1)) return VQS_EINVAL;
  if (options->struct_size != 0 && options->struct_size < sizeof(vqs_options)) return VQS_EINVAL;
  if (max_keys == 0) max_keys = ~0ull;   // the whole batch
  hipStream_t s = (hipStream_t)stream;
  const size_t ks = (size_t)bits / 8;
  // the sample: the longest prefix of segments holding at most max_keys keys (at
  // least one segment), rebased to offset 0
  std::vector<int64_t> h(nseg + 1);
  if (hipMemcpyAsync(h.data(), offsets, (nseg + 1) * sizeof(int64_t), hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    return VQS_EHIP;
  if (h[0] < 0) return VQS_EOFFSETS;
  for (uint64_t i = 0; i < nseg; i++)
    if (h[i + 1] < h[i]) return VQS_EOFFSETS;
  uint64_t k = 1;
  while (k < nseg && (uint64_t)(h[k + 1] - h[0]) <= max_keys) k++;
  const uint64_t sub = (uint64_t)(h[k] - h[0]);
  if (sub == 0) return VQS_OK;
  std::vector<int64_t> rb(k + 1);
  for (uint64_t i = 0; i <= k; i++) rb[i] = h[i] - h[0];
  void* tk = nullptr;
  int64_t* to = nullptr;
  if (hipMalloc(&tk, sub * ks) != hipSuccess || hipMalloc((void**)&to, (k + 1) * sizeof(int64_t)) != hipSuccess) {
    (void)hipGetLastError();
    if (tk) (void)hipFree(tk);
    return VQS_ENOMEM;
  }
  hipEvent_t e0 = nullptr, e1 = nullptr;
  int rc = VQS_OK;
  if (hipMemcpyAsync(to, rb.data(), (k + 1) * sizeof(int64_t), hipMemcpyHostToDevice, s) != hipSuccess ||
      hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
    rc = VQS_EHIP;
  const char* src = (const char*)keys + (size_t)h[0] * ks;
  const uint32_t full = (uint32_t)local_buffer_keys(bits);
  const uint64_t solos[] = {0, 1ull << 14, 1ull << 16, 1ull << 18, 1ull << 20};   // 0: the size rule
  const uint32_t locals[] = {full, full / 2};
  const uint32_t bases[] = {256, 128};
  const uint32_t modes[] = {VQS_LEVEL_LOOKBACK, VQS_LEVEL_RUNS};
  const uint32_t tiles[] = {0, 1};
  float best = -1.0f;
  vqs_options base{};
  std::memcpy(&base, options, sizeof(vqs_options));
  base.struct_size = sizeof(vqs_options);
  base.method = VQS_METHOD_PLAIN;
  base.use_graph = 0;
  vqs_options chosen = base;
  for (uint64_t sm : solos)
    for (uint32_t lk : locals)
      for (uint32_t nb : bases)
        for (uint32_t lm : modes)
          for (uint32_t tv : tiles) {
          if (rc != VQS_OK) break;
          vqs_options c = base;
          c.solo_max = sm;
          c.local_keys = lk;
          c.base_case = nb;
          c.level_mode = lm;
          c.tile_variant = tv;
          float t_min = -1.0f;
          for (int rep = 0; rep < 3 && rc == VQS_OK; rep++) {   // the first run warms up
            if (hipMemcpyAsync(tk, src, sub * ks, hipMemcpyDeviceToDevice, s) != hipSuccess ||
                hipEventRecord(e0, s) != hipSuccess) {
              rc = VQS_EHIP;
              break;
            }
            const int r = sort_impl(tk, to, k, sub, key_type, ascending, &c, s);
            if (r == VQS_EINVAL) break;          // a combination the library rejects
            if (r != VQS_OK) {
              rc = r;
              break;
            }
            float ms = 0.0f;
            if (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
              rc = VQS_EHIP;
              break;
            }
            if (rep > 0 && (t_min < 0.0f || ms < t_min)) t_min = ms;
          }
          if (rc == VQS_OK && t_min >= 0.0f && (best < 0.0f || t_min < best)) {
            best = t_min;
            chosen = c;
          }
        }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  (void)hipStreamSynchronize(s);
  (void)hipFree(tk);
  (void)hipFree(to);
  if (rc != VQS_OK) return rc;
  options->solo_max = chosen.solo_max;
  options->local_keys = chosen.local_keys;
  options->base_case = chosen.base_case;
  options->level_mode = chosen.level_mode;
  options->tile_variant = chosen.tile_variant;
  if (best_ms) *best_ms = best;
  return VQS_OK;
}

int vqs_sort_segmented(void* keys, const int64_t* offsets, uint64_t nseg, int key_type, int ascending) {
  return vqs_sort_segmented_ex(keys, offsets, nseg, key_type, ascending, nullptr, nullptr);
}

uint64_t vqs_workspace_bytes(uint64_t n, uint64_t nseg, int key_type, const vqs_options* options) {
  if (!key_bits(key_type)) return 0;
  std::lock_guard<std::mutex> lock(g_mu);
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) {
    (void)hipGetLastError();
    dev = 0;
  }
  Plan pl;
  if (make_plan(n, nseg ? nseg : 1, key_type, 1, options, geometry(dev), &pl) != VQS_OK) return 0;
  return carve(nullptr, caps_of(pl), nullptr);
}

int vqs_get_stats(void* stream, vqs_stats* out) {
  if (!out) return VQS_EINVAL;
  std::lock_guard<std::mutex> lock(g_mu);
  memset(out, 0, sizeof(*out));
  Workspace* ws = latest_ws((hipStream_t)stream);
  if (!ws || !ws->have_result) return VQS_OK;
  DevStats d;
  if (hipMemcpyAsync(&d, ws->p.stats, sizeof(d), hipMemcpyDeviceToHost, ws->stream) != hipSuccess ||
      hipStreamSynchronize(ws->stream) != hipSuccess)
    return VQS_EHIP;
  out->partitions = d.partitions;
  out->keys_partitioned = d.keys_partitioned;
  out->degenerate = d.degenerate;
  out->all_equal = d.all_equal;
  out->basecases = d.basecases;
  out->fallbacks = d.fallbacks;
  out->fallback_keys = d.fallback_keys;
  out->max_depth = d.max_depth;
  out->level_tiles = d.level_tiles;
  out->solo_items = d.solo_items;
  out->lds_partitions = d.lds_partitions;
  out->hbm_read_keys = d.hbm_read_keys;
  out->hbm_write_keys = d.hbm_write_keys;
  out->bounded_lds = d.bounded_lds;
  out->bounded_global = d.bounded_global;
  // levels that had work
  const int nl = std::min(ws->last_levels + 1, ws->p_levels);
  LevelCtr* h = (LevelCtr*)malloc(sizeof(LevelCtr) * (size_t)std::max(nl, 1));
  if (h && nl > 0 && hipMemcpy(h, ws->p.lvl_ctr, sizeof(LevelCtr) * nl, hipMemcpyDeviceToHost) == hipSuccess) {
    for (int i = 0; i < nl; i++)
      if (h[i].packed) out->levels++;
  }
  free(h);
  if (ws->learned_ran) {
    uint64_t sum[3] = {0, 0, 0};
    float loss = 0.f;
    if (hipMemcpy(sum, ws->l_summary, sizeof(sum), hipMemcpyDeviceToHost) == hipSuccess &&
        hipMemcpy(&loss, ws->l_moments + 2 * MLP_NPARAM, 4, hipMemcpyDeviceToHost) == hipSuccess) {
      out->learned_buckets = NBUCKET;
      out->max_bucket = sum[0];
      out->overflow_buckets = sum[1];
      out->train_loss = loss;
    }
  }
  return VQS_OK;
}

int vqs_learned_fit(const void* keys, uint64_t n, const vqs_options* options, float* params, void* stream) {
  if (!keys || !params || n < 64) return VQS_EINVAL;
  if ((uintptr_t)keys % 8) return VQS_EINVAL;
  std::lock_guard<std::mutex> lock(g_mu);
  Workspace* ws = workspace_for((hipStream_t)stream);
  return learned_locked(ws, const_cast<void*>(keys), n, options, (hipStream_t)stream, true, params);
}

int vqs_mlp_forward(const float* params, const float* x, uint64_t m, float* y, void* stream) {
  if (!params || (m && (!x || !y))) return VQS_EINVAL;
  if (m == 0) return VQS_OK;
  return launch_forward(params, x, m, y, (hipStream_t)stream) == hipSuccess ? VQS_OK : VQS_EHIP;
}

int vqs_mlp_gradient(const float* params, const float* x, const float* t, uint32_t m, float* grad, float* loss,
                     void* stream) {
  if (!params || !x || !t || !grad || !loss || m == 0 || m > (uint32_t)MLP_MAX_BATCH) return VQS_EINVAL;
  return launch_gradient(params, x, t, m, grad, loss, (hipStream_t)stream) == hipSuccess ? VQS_OK : VQS_EHIP;
}

int vqs_mlp_train(float* params, float* moments, const float* x, const float* t, uint64_t m, uint32_t steps,
                  uint32_t batch, float learning_rate, uint64_t sample_seed, int sequential, void* stream) {
  if (!params || !moments || !x || !t || m == 0 || batch == 0 || batch > (uint32_t)MLP_MAX_BATCH) return VQS_EINVAL;
  if (steps == 0) return VQS_OK;
  TrainArgs a{x, t, m, steps, batch, learning_rate, sample_seed, sequential ? 1 : 0};
  return launch_train(params, moments, a, (hipStream_t)stream) == hipSuccess ? VQS_OK : VQS_EHIP;
}

int vqs_mlp_init(float* params, uint64_t model_seed, const float* x, uint64_t m, void* stream) {
  if (!params || !x || m == 0) return VQS_EINVAL;
  return launch_init(params, model_seed, x, m, (hipStream_t)stream) == hipSuccess ? VQS_OK : VQS_EHIP;
}

int vqs_mlp_buckets(const float* params, const uint64_t* keys, uint64_t n, int32_t* out, void* stream) {
  if (!params || (n && (!keys || !out))) return VQS_EINVAL;
  if (n == 0) return VQS_OK;
  return launch_buckets(params, keys, n, out, (hipStream_t)stream) == hipSuccess ? VQS_OK : VQS_EHIP;
}

int vqs_learned_thresholds(const float* params, uint64_t* thresholds, uint32_t* nvalid, void* stream) {
  if (!params || !thresholds || !nvalid) return VQS_EINVAL;
  return launch_thresholds(params, thresholds, nvalid, (hipStream_t)stream) == hipSuccess ? VQS_OK : VQS_EHIP;
}

int vqs_learned_classify(const uint64_t* keys, uint64_t n, const uint64_t* thresholds, const uint32_t* nvalid,
                         int32_t* out, void* stream) {
  if (!thresholds || !nvalid || (n && (!keys || !out))) return VQS_EINVAL;
  if (n == 0) return VQS_OK;
  return launch_classify(keys, n, thresholds, nvalid, out, (hipStream_t)stream) == hipSuccess ? VQS_OK : VQS_EHIP;
}

int vqs_last_error_bits(void* stream, uint32_t* out) {
  if (!out) return VQS_EINVAL;
  std::lock_guard<std::mutex> lock(g_mu);
  *out = 0;
  Workspace* ws = latest_ws((hipStream_t)stream);
  if (!ws || !ws->p.err) return VQS_OK;
  unsigned int e = 0;
  if (hipMemcpyAsync(&e, ws->p.err, 4, hipMemcpyDeviceToHost, ws->stream) != hipSuccess ||
      hipStreamSynchronize(ws->stream) != hipSuccess)
    return VQS_EHIP;
  *out = e;
  return VQS_OK;
}

int vqs_profile(int enable) {
  if (enable < 0 || enable > 2) return VQS_EINVAL;
  std::lock_guard<std::mutex> lock(g_mu);
  g_profile = enable;
  return VQS_OK;
}

int vqs_profile_read(void* stream, vqs_kernel_time* out, int max, int* count) {
  if (!count || (max > 0 && !out)) return VQS_EINVAL;
  std::lock_guard<std::mutex> lock(g_mu);
  *count = 0;
  auto it = g_ws.find(std::make_pair(current_device(), (hipStream_t)stream));
  if (it == g_ws.end() || !it->second->p.lvl_ctr) return VQS_OK;
  Workspace* ws = it->second.get();
  if (hipStreamSynchronize(ws->stream) != hipSuccess) return VQS_EHIP;
  std::vector<LevelCtr> ctr((size_t)ws->p_levels);
  if (hipMemcpy(ctr.data(), ws->p.lvl_ctr, sizeof(LevelCtr) * ctr.size(), hipMemcpyDeviceToHost) != hipSuccess)
    return VQS_EHIP;
  int n = 0;
  for (const ProfRec& r : ws->prof) {
    if (n >= max) break;
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, r.a, r.b) != hipSuccess) return VQS_EHIP;
    out[n].kind = r.kind;
    out[n].level = r.level;
    out[n].keys = (r.kind == 2 && r.level >= 0 && r.level < (int)ctr.size()) ? ctr[r.level].keys : 0;
    out[n].ms = ms;
    n++;
  }
  *count = n;
  ws->prof.clear();
  ws->events_used = 0;
  return VQS_OK;
}

int vqs_release(void) {
  std::lock_guard<std::mutex> lock(g_mu);
  for (auto& kv : g_ws) (void)hipStreamSynchronize(kv.second->stream);
  g_ws.clear();
  return VQS_OK;
}

const char* vqs_strerror(int code) {
  switch (code) {
    case VQS_OK: return "success";
    case VQS_EINVAL: return "invalid argument";
    case VQS_ETYPE: return "unknown key type";
    case VQS_ENOMEM: return "device workspace allocation failed";
    case VQS_EHIP: return "HIP runtime error";
    case VQS_EOFFSETS: return "segment offsets decrease";
    case VQS_EINTERNAL: return "device-side capacity check failed";
    case VQS_ESIZE: return "input larger than the fixed scratch of vqs_sort_noalloc allows";
    default: return "unknown error";
  }
}

int vqs_version(void) { return VERSION; }


}  // extern "C"
