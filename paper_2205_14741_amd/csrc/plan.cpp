// Symbolic plan of the submatrix method (host), step 1 of Fig. 2 of the paper:
// index sets, submatrix sizes, the offset of every atom's own columns, padding,
// processing order, chunking of the workspace, and the device copies of these
// tables.
#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>

#include "plan.h"

namespace sm {

static thread_local std::string g_last_error;

int set_error(int code, const char* fmt, ...) {
  char buf[1024];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return code;
}

int hip_error(hipError_t e, const char* what) {
  return set_error(SM_ERR_HIP, "HIP error %d (%s) in %s", (int)e, hipGetErrorString(e), what);
}

int storage_is_f64(const sm_sign_opts* o) {
  if (o->phase1 == SM_F64) return 1;
  if (o->refine_steps > 0 && o->refine == SM_F64) return 1;
  return 0;
}

// Workspace storage of a schedule: SM_F64 or SM_F32 for the iterate's type,
// or the main precision (SM_BF16 / SM_F16 / SM_BF16X3) for float32 buffers
// each paired with the operand copy its matrix-core products read.
int ws_storage(const sm_sign_opts* o) {
  if (storage_is_f64(o)) return SM_F64;
  if (o->phase1 == SM_BF16 || o->phase1 == SM_F16 || o->phase1 == SM_BF16X3) return o->phase1;
  return SM_F32;
}

bool valid_storage(int storage) { return storage >= SM_F64 && storage <= SM_BF16X3; }

static_assert(sizeof(sm_sign_opts) == 104, "sm_sign_opts layout");
static_assert(sizeof(sm_sub_stats) == 152, "sm_sub_stats layout");

static int64_t align256(int64_t x) { return (x + 255) & ~int64_t(255); }

}  // namespace sm

using namespace sm;

sm::WsLayout sm_plan::layout(int storage) const {
  WsLayout L{};
  // float64 iterates, or float32 ones followed by a region of operand copies
  // of the same size (2 bf16 / f16 planes or one, in a float32 slot each)
  const int64_t es = storage == SM_F32 ? 4 : 8;
  int64_t off = 0;
  L.mats = off;
  off = align256(off + max_mats * es);
  L.state = off;
  off = align256(off + max_subs * (int64_t)sizeof(SubState));
  L.partials = off;
  off = align256(off + max_tiles * 8);
  L.lists = off;
  // 4 lists: count_tiles, count_subs, list[max_subs], prefix[max_subs+1]
  off = align256(off + 4 * (2 + max_subs + max_subs + 1) * 4 + 64);
  L.tiles = off;
  off = align256(off + 4 * max_tiles * (int64_t)sizeof(TileRec));
  L.features = off;
  off = align256(off + max_subs * kNumFeatures * 4);
  L.scratch = off;
  off = align256(off + max_subs * 8 * 8);
  L.vecs = off;
  off = align256(off + max_vecs * 8);
  L.flag = off;
  off = align256(off + 256);
  L.total = off;
  return L;
}

extern "C" {

const char* sm_last_error(void) { return g_last_error.c_str(); }

const char* sm_version(void) { return "smsign 0.1 (gfx950)"; }

int sm_default_opts(int32_t prec, sm_sign_opts* o) {
  if (!o) return set_error(SM_ERR_ARG, "sm_default_opts: null opts");
  if (prec < SM_F64 || prec > SM_BF16X3) return set_error(SM_ERR_ARG, "sm_default_opts: bad precision %d", prec);
  std::memset(o, 0, sizeof(*o));
  o->phase1 = prec;
  o->refine = SM_F32;
  o->max_iter = 100;
  o->tol = 1e-10;
  o->switch_tol = 0.1;
  o->stall_below = 0.5;
  o->stall_ratio = 0.8;
  o->scaling = SM_SCALE_GERSHGORIN;
  o->power_steps = 8;
  o->scale_margin = 0.05;
  o->probes = 2;
  o->variant = -1;
  o->graph_iters = 0;
  o->retry = 1;
  if (prec == SM_F64) {
    o->refine_steps = 0;
    o->refine = SM_F64;
  } else if (prec == SM_F32) {
    o->refine_steps = 0;
    o->tol = 1e-10;          // not reachable in float32: the stagnation test stops it
    o->stall_below = 1e-2;
    o->stall_ratio = 0.5;
  } else {
    o->refine_steps = (prec == SM_BF16) ? 3 : 2;
  }
  return SM_OK;
}

}  // extern "C"

namespace {

// Processing order -> the order-dependent tables: per processing index g the
// submatrix, its padded size and offsets inside its chunk; chunks fill the
// element budget in processing order (a larger submatrix forms its own);
// every chunk's size class (256-row tiles of its largest submatrix) and the
// default GEMM variants of every class until sm_autotune measures better
// ones: the XCD-aware 64-wide tiles for float64 and small submatrices, the
// 256-wide tiles with synchronized rounds for the 16-bit precisions on large
// ones (their float32 refinement on the 128-wide ring kernel), the half-depth
// stages on plans padded to 32.
void assign_order(sm_plan* p, const std::vector<int32_t>& order) {
  const int32_t n = p->n_atoms;
  p->order_g.assign(order.begin(), order.end());
  p->npad_g.assign(n, 0);
  p->mat_off_g.assign(n, 0);
  p->tile_off_g.assign(n, 0);
  p->vec_off_g.assign(n, 0);
  p->chunk_of.assign(n, 0);
  p->chunk_ptr.assign(1, 0);
  p->chunk_class.clear();
  p->max_mats = p->max_tiles = p->max_vecs = p->max_subs = 0;
  int64_t mats = 0, tiles = 0, vecs = 0, subs = 0;
  int32_t chunk_max = 0;
  std::vector<int32_t> class_max(kMaxClasses, 0);   // largest n_pad of every class
  auto close_chunk = [&]() {
    const int32_t c = (chunk_max + kClassRows - 1) / kClassRows;
    p->chunk_class.push_back(c);
    class_max[c] = std::max(class_max[c], chunk_max);
  };
  for (int32_t g = 0; g < n; ++g) {
    const int32_t i = order[g];
    const int64_t np = p->npad[i];
    const int64_t need = 3 * np * np;
    const int64_t T = tiles_of((int)np);
    const int64_t nt = T * (T + 1) / 2;
    if (subs > 0 && p->max_chunk_elems > 0 && mats + need > p->max_chunk_elems) {
      close_chunk();
      p->chunk_ptr.push_back(g);
      mats = tiles = vecs = subs = 0;
      chunk_max = 0;
    }
    p->npad_g[g] = (int32_t)np;
    p->mat_off_g[g] = mats;
    p->tile_off_g[g] = (int32_t)tiles;
    p->vec_off_g[g] = vecs;
    p->chunk_of[i] = (int32_t)p->chunk_ptr.size() - 1;
    chunk_max = std::max(chunk_max, (int32_t)np);
    mats += need;
    tiles += nt;
    vecs += np * 2 * kMaxProbes;
    subs += 1;
    p->max_mats = std::max(p->max_mats, mats);
    p->max_tiles = std::max(p->max_tiles, tiles);
    p->max_vecs = std::max(p->max_vecs, vecs);
    p->max_subs = std::max(p->max_subs, subs);
  }
  close_chunk();
  p->chunk_ptr.push_back(n);
  auto defaults = [&](int32_t largest, int32_t* t) {
    const bool big = p->pad_to >= 64 && largest >= 768;
    t[SM_F64] = 1;
    t[SM_F32] = big ? 5 : 1;
    for (int m : {SM_BF16, SM_F16, SM_BF16X3}) t[m] = p->pad_to < 64 ? 2 : big ? 8 : 1;
  };
  defaults(p->max_npad, p->tuned);
  p->class_tuned.assign(kMaxClasses, {-1, -1, -1, -1, -1});
  for (int32_t c : p->chunk_class) defaults(class_max[c], p->class_tuned[c].data());
}

// Morton (Z-order) key of a point inside [lo, lo + span)^3, 21 bits per axis.
uint64_t morton3(const double* x, const double* lo, double span) {
  uint64_t key = 0;
  uint32_t q[3];
  for (int d = 0; d < 3; ++d) {
    const double t = span > 0 ? (x[d] - lo[d]) / span : 0.0;
    const double c = std::min(std::max(t, 0.0), 1.0) * 2097151.0;
    q[d] = (uint32_t)c;
  }
  for (int b = 20; b >= 0; --b)
    for (int d = 0; d < 3; ++d) key = (key << 1) | ((q[d] >> b) & 1u);
  return key;
}

}  // namespace

extern "C" {

int sm_plan_set_positions(sm_plan* p, const double* xyz, int32_t bucket_rows) {
  if (!p || !xyz) return set_error(SM_ERR_ARG, "sm_plan_set_positions: null argument");
  if (p->device >= 0)
    return set_error(SM_ERR_STATE, "sm_plan_set_positions: the plan has already been used on a device");
  const int32_t n = p->n_atoms;
  double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
  for (int32_t i = 0; i < n; ++i)
    for (int d = 0; d < 3; ++d) {
      const double v = xyz[3 * (int64_t)i + d];
      if (!std::isfinite(v)) return set_error(SM_ERR_ARG, "sm_plan_set_positions: position of atom %d is not finite", i);
      lo[d] = std::min(lo[d], v);
      hi[d] = std::max(hi[d], v);
    }
  const double span = std::max({hi[0] - lo[0], hi[1] - lo[1], hi[2] - lo[2]}) * (1.0 + 1e-12);
  struct Key {
    int32_t bucket;
    uint64_t z;
    int32_t i;
  };
  std::vector<Key> keys(n);
  for (int32_t i = 0; i < n; ++i)
    keys[i] = Key{bucket_rows > 0 ? p->npad[i] / bucket_rows : 0, morton3(xyz + 3 * (int64_t)i, lo, span), i};
  // larger size buckets first, Morton order inside a bucket, atom id on ties
  std::sort(keys.begin(), keys.end(), [](const Key& a, const Key& b) {
    if (a.bucket != b.bucket) return a.bucket > b.bucket;
    if (a.z != b.z) return a.z < b.z;
    return a.i < b.i;
  });
  std::vector<int32_t> order(n);
  for (int32_t g = 0; g < n; ++g) order[g] = keys[g].i;
  assign_order(p, order);
  return SM_OK;
}

int sm_plan_create(const sm_bsr_pattern* pat, int32_t pad_to, int64_t max_chunk_elems,
                   sm_plan** out) {
  if (!pat || !out) return set_error(SM_ERR_ARG, "sm_plan_create: null argument");
  *out = nullptr;
  if (pat->n_atoms <= 0) return set_error(SM_ERR_ARG, "sm_plan_create: n_atoms must be > 0");
  if (!pat->block_size || !pat->col_ptr || !pat->row_idx || !pat->panel_off)
    return set_error(SM_ERR_ARG, "sm_plan_create: null pattern array");
  if (pad_to != 32 && pad_to != 64 && pad_to != 128)
    return set_error(SM_ERR_ARG, "sm_plan_create: pad_to must be 32, 64 or 128 (got %d)", pad_to);
  const int32_t n = pat->n_atoms;
  if (pat->col_ptr[0] != 0) return set_error(SM_ERR_ARG, "sm_plan_create: col_ptr[0] != 0");
  for (int32_t c = 0; c < n; ++c) {
    if (pat->block_size[c] < 1) return set_error(SM_ERR_ARG, "sm_plan_create: block_size[%d] < 1", c);
    if (pat->col_ptr[c + 1] <= pat->col_ptr[c])
      return set_error(SM_ERR_ARG, "sm_plan_create: block column %d is empty (diagonal missing)", c);
  }
  sm_plan* p = new (std::nothrow) sm_plan();
  if (!p) return set_error(SM_ERR_OOM, "sm_plan_create: out of host memory");
  p->n_atoms = n;
  p->nnzb = pat->col_ptr[n];
  p->bs.assign(pat->block_size, pat->block_size + n);
  p->col_ptr.assign(pat->col_ptr, pat->col_ptr + n + 1);
  p->row_idx.assign(pat->row_idx, pat->row_idx + p->nnzb);
  p->panel_off.assign(pat->panel_off, pat->panel_off + n + 1);
  p->pad_to = pad_to;
  p->blk_rowoff.resize(p->nnzb);
  p->height.resize(n);
  p->loc.resize(n);
  p->npad.resize(n);
  int64_t N = 0;
  for (int32_t c = 0; c < n; ++c) N += p->bs[c];
  p->diag_idx.resize(N);

  if (p->panel_off[0] != 0) { delete p; return set_error(SM_ERR_ARG, "sm_plan_create: panel_off[0] != 0"); }
  int64_t dpos = 0;
  for (int32_t c = 0; c < n; ++c) {
    int64_t k0 = p->col_ptr[c], k1 = p->col_ptr[c + 1];
    int32_t h = 0;
    int32_t loc = -1;
    int32_t prev = -1;
    for (int64_t k = k0; k < k1; ++k) {
      int32_t r = p->row_idx[k];
      if (r < 0 || r >= n) { delete p; return set_error(SM_ERR_ARG, "sm_plan_create: row index %d out of range in column %d", r, c); }
      if (r <= prev) { delete p; return set_error(SM_ERR_ARG, "sm_plan_create: rows of block column %d are not strictly ascending", c); }
      prev = r;
      p->blk_rowoff[k] = h;
      if (r == c) loc = h;
      h += p->bs[r];
    }
    if (loc < 0) { delete p; return set_error(SM_ERR_ARG, "sm_plan_create: diagonal block of column %d missing", c); }
    if (h > 32767) {
      delete p;
      return set_error(SM_ERR_ARG, "sm_plan_create: block column %d has %d rows; at most 32767 are supported", c, h);
    }
    p->height[c] = h;
    p->loc[c] = loc;
    p->npad[c] = (int32_t)((h + pad_to - 1) / pad_to * pad_to);
    if ((int64_t)h * p->bs[c] != p->panel_off[c + 1] - p->panel_off[c]) {
      const int32_t w = p->bs[c];
      delete p;
      return set_error(SM_ERR_ARG, "sm_plan_create: panel_off of column %d does not match height %d x width %d",
                       c, h, w);
    }
    for (int32_t q = 0; q < p->bs[c]; ++q)
      p->diag_idx[dpos++] = p->panel_off[c] + (int64_t)q * h + loc + q;
    p->max_m = std::max<int32_t>(p->max_m, (int32_t)(k1 - k0));
    p->max_npad = std::max(p->max_npad, p->npad[c]);
  }
  p->nvals = p->panel_off[n];
  // structural symmetry: every stored (r, c) has (c, r)
  for (int32_t c = 0; c < n; ++c) {
    for (int64_t k = p->col_ptr[c]; k < p->col_ptr[c + 1]; ++k) {
      int32_t r = p->row_idx[k];
      const int32_t* b = p->row_idx.data() + p->col_ptr[r];
      const int32_t* e = p->row_idx.data() + p->col_ptr[r + 1];
      if (!std::binary_search(b, e, c)) {
        delete p;
        return set_error(SM_ERR_ARG, "sm_plan_create: pattern not symmetric: block (%d,%d) stored, (%d,%d) not",
                         r, c, c, r);
      }
    }
  }
  p->max_chunk_elems = max_chunk_elems;
  std::vector<int32_t> order(n);
  for (int32_t g = 0; g < n; ++g) order[g] = g;
  assign_order(p, order);
  *out = p;
  return SM_OK;
}

void sm_plan_destroy(sm_plan* p) {
  if (!p) return;
  if (p->device >= 0) {
    int cur = -1;
    (void)hipGetDevice(&cur);
    (void)hipSetDevice(p->device);
    for (void* a : p->dev_allocs) (void)hipFree(a);
    if (p->h_pinned) (void)hipHostFree(p->h_pinned);
    for (auto& e : p->ev)
      if (e) (void)hipEventDestroy(e);
    for (auto& e : p->prof_ev) (void)hipEventDestroy(e);
    for (auto& g : p->graphs) (void)hipGraphExecDestroy(g.exec);
    if (p->capture_stream) (void)hipStreamDestroy(p->capture_stream);
    if (cur >= 0) (void)hipSetDevice(cur);
  }
  delete p;
}

int sm_ws_storage(const sm_sign_opts* o) { return o ? ws_storage(o) : -1; }

int sm_plan_sizes(const sm_plan* p, int32_t storage_prec, int64_t* n_sub, int64_t* n_chunks,
                  int64_t* ws_bytes, int64_t* p_nnz_vals) {
  if (!p) return set_error(SM_ERR_ARG, "sm_plan_sizes: null plan");
  if (!valid_storage(storage_prec))
    return set_error(SM_ERR_ARG, "sm_plan_sizes: bad storage code %d", storage_prec);
  if (n_sub) *n_sub = p->n_atoms;
  if (n_chunks) *n_chunks = (int64_t)p->chunk_ptr.size() - 1;
  if (ws_bytes) *ws_bytes = p->layout(storage_prec).total;
  if (p_nnz_vals) *p_nnz_vals = p->nvals;
  return SM_OK;
}

int sm_plan_info(const sm_plan* p, int32_t* n_out, int32_t* npad_out, int32_t* loc_out,
                 int32_t* chunk_out, int32_t* order_out) {
  if (!p) return set_error(SM_ERR_ARG, "sm_plan_info: null plan");
  const size_t n = p->n_atoms;
  if (n_out) std::memcpy(n_out, p->height.data(), n * 4);
  if (npad_out) std::memcpy(npad_out, p->npad.data(), n * 4);
  if (loc_out) std::memcpy(loc_out, p->loc.data(), n * 4);
  if (chunk_out) std::memcpy(chunk_out, p->chunk_of.data(), n * 4);
  if (order_out) std::memcpy(order_out, p->order_g.data(), n * 4);
  return SM_OK;
}

}  // extern "C"

namespace sm {

template <typename T>
static int upload(sm_plan* p, const std::vector<T>& v, const T** dst) {
  void* d = nullptr;
  size_t bytes = std::max<size_t>(v.size() * sizeof(T), 16);
  hipError_t e = hipMalloc(&d, bytes);
  if (e != hipSuccess) return set_error(SM_ERR_OOM, "plan upload: hipMalloc(%zu) failed: %s", bytes, hipGetErrorString(e));
  p->dev_allocs.push_back(d);
  if (!v.empty()) SM_HIP(hipMemcpy(d, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice));
  *dst = (const T*)d;
  return SM_OK;
}

template <typename T>
static int dev_alloc(sm_plan* p, size_t count, T** dst) {
  void* d = nullptr;
  hipError_t e = hipMalloc(&d, std::max<size_t>(count * sizeof(T), 16));
  if (e != hipSuccess) return set_error(SM_ERR_OOM, "plan: hipMalloc failed: %s", hipGetErrorString(e));
  p->dev_allocs.push_back(d);
  *dst = (T*)d;
  return SM_OK;
}

int ensure_device(sm_plan* p) {
  int dev = -1;
  SM_HIP(hipGetDevice(&dev));
  if (p->device >= 0) {
    if (dev != p->device)
      return set_error(SM_ERR_STATE, "plan was first used on device %d, now device %d is current", p->device, dev);
    return SM_OK;
  }
  int rc;
  DevPlan& d = p->dev;
#define UP(vec, field) \
  if ((rc = upload(p, p->vec, &d.field)) != SM_OK) return rc;
  UP(bs, bs);
  UP(col_ptr, col_ptr);
  UP(row_idx, row_idx);
  UP(panel_off, panel_off);
  UP(blk_rowoff, blk_rowoff);
  UP(height, height);
  UP(loc, loc);
  UP(order_g, order_g);
  UP(npad_g, npad_g);
  UP(mat_off_g, mat_off_g);
  UP(tile_off_g, tile_off_g);
  UP(vec_off_g, vec_off_g);
#undef UP
  const int64_t* di = nullptr;
  if ((rc = upload(p, p->diag_idx, &di)) != SM_OK) return rc;
  p->d_diag_idx = const_cast<int64_t*>(di);
  if ((rc = dev_alloc(p, 2 * kTraceBlocks + 8, &p->d_trace_parts)) != SM_OK) return rc;
  if ((rc = dev_alloc(p, (size_t)p->n_atoms, &p->d_ne_sub)) != SM_OK) return rc;
  if ((rc = dev_alloc(p, (size_t)2 * p->n_atoms, &p->d_gersh)) != SM_OK) return rc;
  // coherent and mapped: the scheduler writes the live count straight into it
  SM_HIP(hipHostMalloc((void**)&p->h_pinned, kHostWords * 4, hipHostMallocMapped | hipHostMallocCoherent));
  std::memset(p->h_pinned, 0, kHostWords * 4);
  SM_HIP(hipHostGetDevicePointer((void**)&p->d_pinned, p->h_pinned, 0));
  int ncu = 0;
  if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && ncu > 0)
    p->num_cu = ncu;
  SM_HIP(hipEventCreateWithFlags(&p->ev[0], hipEventDisableTiming));
  SM_HIP(hipEventCreateWithFlags(&p->ev[1], hipEventDisableTiming));
  p->device = dev;
  return SM_OK;
}

}  // namespace sm
