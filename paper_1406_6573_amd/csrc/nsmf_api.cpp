// C ABI of the engine: context, mesh upload and validation, parameters, state, and the
// residual / Jacobian-apply / VJP entry points declared in include/nsmf.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/nsmf.h"
#include "nsmf_internal.h"

using namespace nsmf;

namespace {

template <typename T> struct DevBuf {
  T *p = nullptr;
  size_t n = 0;
  hipError_t alloc(size_t count) {
    free();
    n = count;
    if (count == 0) return hipSuccess;
    return hipMalloc((void **)&p, count * sizeof(T));
  }
  void free() {
    if (p) (void)hipFree(p);
    p = nullptr;
    n = 0;
  }
};

// Scratch of the allocation-free Jacobian apply (nsmf_jacobian_apply_noalloc): the element vector
// (per-node partial sums) of one apply lives in this file-scope device array instead of the
// context's allocation.  Every device that loads the library holds its own copy, at its own
// address, until the process ends.  Host code never passes the array's name to a kernel (on the
// host it is only a stand-in symbol): the device address is looked up once per device with
// hipGetSymbolAddress in nsmf_create, with that device current, and kept in scratch_ptr.
constexpr size_t NOALLOC_SCRATCH_BYTES = size_t(64) << 20;
__device__ __align__(256) unsigned char scratch[NOALLOC_SCRATCH_BYTES];
constexpr int MAX_DEVICES = 64;
std::mutex scratch_mutex;
void *scratch_ptr[MAX_DEVICES] = {};

// Device address of the scratch array on the current device (hip_device), looked up on the
// first call for that device.
hipError_t scratch_address(int hip_device, void **out) {
  std::lock_guard<std::mutex> lock(scratch_mutex);
  if (hip_device < 0 || hip_device >= MAX_DEVICES) return hipErrorInvalidDevice;
  if (scratch_ptr[hip_device] == nullptr) {
    void *ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    scratch_ptr[hip_device] = ptr;
  }
  *out = scratch_ptr[hip_device];
  return hipSuccess;
}

int launch_threads(int P) { return P == 5 ? Launch<5>::NT : (P == 4 ? Launch<4>::NT : Launch<3>::NT); }
int launch_elems(int P) { return P == 5 ? Launch<5>::E : (P == 4 ? Launch<4>::E : Launch<3>::E); }

}  // namespace

struct nsmf_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  void *scratch = nullptr;   // this device's address of the allocation-free apply's scratch array
  std::string err = "";
  // mesh
  bool have_mesh = false;
  int k = 0, P = 0, n_p = 0, ps = PS_P, geo = GEO_AFFINE, nt = 0, epb = 0, nblocks = 0, any_hang = 0;
  int64_t n_el = 0, n_nodes = 0, n_bface = 0, n_inc = 0, n_ent = 0;
  HostTables tab;
  DevBuf<uint32_t> en, cmask;
  DevBuf<int32_t> bface_of, inc_ptr;   // node -> first entry of its segment of the element vector
  DevBuf<int32_t> pos;                // P = 4: element slot -> its entry in the element vector
  DevBuf<int32_t> spos;               // P = 3, 5, per block: element-vector entries of its slots, ascending
  DevBuf<uint16_t> sslot;             // per block: LDS staging index of each of those slots
  DevBuf<uint8_t> dmask;
  DevBuf<double> tabs;                // TabSet<P> of the mesh's degree
  DevBuf<double> geo_el64, geo_qp64, face64;
  DevBuf<float> geo_el32, geo_qp32, face32;
  DevBuf<int32_t> rot_of;             // element -> row of its bottom-slot frames, -1 (nodal frames)
  DevBuf<double> rot64;
  DevBuf<float> rot32;
  // params
  bool have_params = false;
  nsmf_params prm;
  int lin = NSMF_NEWTON;
  DevBuf<double> logA, beta64;
  DevBuf<float> beta32;
  // state
  bool have_state = false;
  DevBuf<double> st64, fst64, u, p, ev;   // ev: element vector (double or float)
  DevBuf<float> st32, fst32;
  // Krylov vector kernels: partial sums of the multi-dot products
  DevBuf<double> dot_partial;
  // low-order approximation F~: node coordinates (kept from upload), periodic translations, and the
  // nodal data of the current state (computed on first use after set_state)
  DevBuf<double> xyz, lo;
  double period[3] = {0.0, 0.0, 0.0};
  bool have_lo = false;
  bool has_frames = false;
  // horizontal coarse space of the two-level velocity preconditioner: per node its coarse cell's corner
  // points and bilinear weights and its relative height; per coarse point the list of its nodes
  int64_t n_cpts = 0;
  DevBuf<int32_t> c_cpt, c_node;
  DevBuf<double> c_w, c_zeta, c_wt;
  DevBuf<int64_t> c_ptr;
  // vertical node lines of the line-block preconditioner: chains of nodes linked through the
  // conforming z-lines of the elements (host arrays built at upload, copied at the first setup)
  bool lines_ok = false, have_lines = false;
  int64_t n_lines = 0;
  std::vector<int32_t> h_line_ptr, h_line_node, h_lptr, h_lslot;
  DevBuf<int32_t> line_ptr, line_node, line_prow, line_row, line_first, lptr, lslot;
  int64_t line_nr = 0;   // line-block rows per component (interleaved groups, padded)
  DevBuf<double> lbuf, lfac64;
  DevBuf<float> lfac32;
  // timing
  bool timing = false;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> events;

  int fail(int code, const std::string &msg) {
    err = msg;
    return code;
  }
  int hip(hipError_t e, const char *what) {
    if (e == hipSuccess) return NSMF_OK;
    err = std::string(what) + ": " + hipGetErrorString(e);
    return e == hipErrorOutOfMemory ? NSMF_ENOMEM : NSMF_EHIP;
  }
  MeshView mesh_view() const {
    MeshView m;
    m.en = en.p;
    m.cmask = cmask.p;
    m.bface_of = bface_of.p;
    m.rot_of = rot_of.p;
    m.pos = pos.p;
    m.spos = spos.p;
    m.sslot = sslot.p;
    m.n_inc = n_inc;
    m.n_ent = n_ent;
    m.n_el = n_el;
    m.n_nodes = n_nodes;
    m.nblocks = nblocks;
    m.any_hang = any_hang;
    return m;
  }
  GeoView<double> geo64() const { return GeoView<double>{geo_el64.p, geo_qp64.p, face64.p, rot64.p}; }
  GeoView<float> geo32() const { return GeoView<float>{geo_el32.p, geo_qp32.p, face32.p, rot32.p}; }
  void free_mesh() {
    en.free(); cmask.free(); bface_of.free(); inc_ptr.free(); pos.free(); spos.free(); sslot.free(); dmask.free(); ev.free(); tabs.free();
    geo_el64.free(); geo_qp64.free(); face64.free(); geo_el32.free(); geo_qp32.free(); face32.free();
    rot_of.free(); rot64.free(); rot32.free();
    logA.free(); beta64.free(); beta32.free();
    st64.free(); fst64.free(); u.free(); p.free(); st32.free(); fst32.free(); dot_partial.free();
    xyz.free(); lo.free();
    have_lo = false;
    has_frames = false;
    c_cpt.free(); c_node.free(); c_w.free(); c_zeta.free(); c_wt.free(); c_ptr.free();
    n_cpts = 0;
    line_ptr.free(); line_node.free(); line_prow.free(); line_row.free(); line_first.free(); lptr.free(); lslot.free();
    lbuf.free(); lfac64.free(); lfac32.free();
    line_nr = 0;
    h_line_ptr.clear(); h_line_node.clear(); h_lptr.clear(); h_lslot.clear();
    lines_ok = have_lines = false;
    n_lines = 0;
    have_mesh = have_params = have_state = false;
  }
};

#define NSMF_TRY(ctx, expr, what)                    \
  do {                                               \
    int _rc = (ctx)->hip((expr), (what));            \
    if (_rc != NSMF_OK) return _rc;                  \
  } while (0)

extern "C" {

const char *nsmf_version(void) { return "nsmf 0.1 (gfx950)"; }

const char *nsmf_last_error(const nsmf_ctx *ctx) { return ctx ? ctx->err.c_str() : "null context"; }

int nsmf_create(nsmf_ctx **out, int hip_device) {
  if (!out) return NSMF_EINVAL;
  *out = nullptr;
  int n = 0;
  if (hipGetDeviceCount(&n) != hipSuccess || hip_device < 0 || hip_device >= n) return NSMF_EINVAL;
  if (hipSetDevice(hip_device) != hipSuccess) return NSMF_EHIP;
  void *scr = nullptr;
  if (scratch_address(hip_device, &scr) != hipSuccess || scr == nullptr) return NSMF_EHIP;
  nsmf_ctx *c = new nsmf_ctx();
  c->device = hip_device;
  c->scratch = scr;
  *out = c;
  return NSMF_OK;
}

void nsmf_destroy(nsmf_ctx *ctx) {
  if (!ctx) return;
  (void)hipSetDevice(ctx->device);
  (void)hipStreamSynchronize(ctx->stream);
  for (auto &ev : ctx->events) {
    (void)hipEventDestroy(ev.first);
    (void)hipEventDestroy(ev.second);
  }
  ctx->free_mesh();
  delete ctx;
}

int nsmf_set_stream(nsmf_ctx *ctx, void *stream) {
  if (!ctx) return NSMF_EINVAL;
  ctx->stream = (hipStream_t)stream;
  return NSMF_OK;
}

int nsmf_upload_mesh(nsmf_ctx *ctx, const nsmf_mesh *m) {
  if (!ctx || !m) return NSMF_EINVAL;
  NSMF_TRY(ctx, hipSetDevice(ctx->device), "hipSetDevice");
  if (m->k < 2 || m->k > 4) return ctx->fail(NSMF_EUNSUP, "k must be 2, 3 or 4");
  if (m->pspace != PS_P && m->pspace != PS_Q) return ctx->fail(NSMF_EINVAL, "pspace must be 0 (P_{k-1}) or 1 (Q_{k-2})");
  if (m->n_el <= 0 || m->n_nodes <= 0 || m->n_bface < 0) return ctx->fail(NSMF_EINVAL, "sizes must be positive");
  if (m->n_nodes >= (int64_t)NODE_MASK) return ctx->fail(NSMF_EINVAL, "n_nodes must be below 2^28");
  if (!m->elem_nodes || !m->cmask || !m->coords || (m->n_bface > 0 && !m->bface_elem))
    return ctx->fail(NSMF_EINVAL, "NULL mesh array");
  for (int d = 0; d < 2; ++d)
    if (!(m->period[d] >= 0.0) || !std::isfinite(m->period[d]))
      return ctx->fail(NSMF_EINVAL, "period must be finite and >= 0");
  if (m->period[2] != 0.0) return ctx->fail(NSMF_EUNSUP, "periodic z axis");
  ctx->free_mesh();
  const int P = m->k + 1, P2 = P * P, P3 = P2 * P;
  const int64_t n_el = m->n_el, N = m->n_nodes, NB = m->n_bface;
  // ---- host validation and node words
  std::vector<uint32_t> words((size_t)n_el * P3);
  for (int64_t i = 0; i < n_el * P3; ++i) {
    const int32_t id = m->elem_nodes[i];
    if (id < 0 || id >= N) return ctx->fail(NSMF_EMESH, "elem_nodes entry out of range");
    uint32_t wd = (uint32_t)id;
    if (m->dmask)
      for (int c = 0; c < 3; ++c)
        if (m->dmask[c * N + id]) wd |= 1u << (MASK_SHIFT + c);
    words[i] = wd;
  }
  int any_hang = 0;
  for (int64_t e = 0; e < n_el; ++e) {
    if (m->cmask[e] >> 21) return ctx->fail(NSMF_EMESH, "cmask has bits above 20");
    if (m->cmask[e] >> 3) any_hang = 1;
  }
  // ---- nodal frames: orthonormal, each node once, named only by bottom slots (z = 0)
  std::vector<int32_t> frame_row;
  if (m->n_frames < 0 || (m->n_frames > 0 && (!m->frame_nodes || !m->frames)))
    return ctx->fail(NSMF_EINVAL, "n_frames < 0 or NULL frame arrays");
  if (m->n_frames > 0) {
    frame_row.assign((size_t)N, -1);
    for (int64_t f = 0; f < m->n_frames; ++f) {
      const int32_t id = m->frame_nodes[f];
      if (id < 0 || id >= N) return ctx->fail(NSMF_EMESH, "frame_nodes entry out of range");
      if (frame_row[id] >= 0) return ctx->fail(NSMF_EMESH, "node listed twice in frame_nodes");
      frame_row[id] = (int32_t)f;
      const double *Q = m->frames + 9 * f;
      for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) {
          const double d = Q[a] * Q[b] + Q[3 + a] * Q[3 + b] + Q[6 + a] * Q[6 + b];   // (Q^T Q)_ab
          if (!(std::fabs(d - (a == b ? 1.0 : 0.0)) <= 1e-12)) return ctx->fail(NSMF_EMESH, "frame not orthonormal");
        }
    }
    for (int64_t i = 0; i < n_el * P3; ++i)
      if (frame_row[words[i] & NODE_MASK] >= 0) {
        if ((i % P3) / P2 != 0) return ctx->fail(NSMF_EMESH, "node with a frame in a slot above the bottom");
        words[i] |= ROT_BIT;
      }
  }
  std::vector<int32_t> bof((size_t)n_el, -1);
  for (int64_t f = 0; f < NB; ++f) {
    const int32_t e = m->bface_elem[f];
    if (e < 0 || e >= n_el) return ctx->fail(NSMF_EMESH, "bface_elem entry out of range");
    if (bof[e] >= 0) return ctx->fail(NSMF_EMESH, "element listed twice in bface_elem");
    bof[e] = (int32_t)f;
  }
  std::vector<uint8_t> dm((size_t)3 * N, 0);
  if (m->dmask)
    for (int64_t i = 0; i < 3 * N; ++i) dm[i] = m->dmask[i] ? 1 : 0;
  if (3 * N >= (int64_t)0x7FFFFFFF) return ctx->fail(NSMF_EINVAL, "3*n_nodes must fit in int32");
  // ---- vertical node lines (line-block preconditioner): node n links to the node above it
  // through every z-line of an element on which neither of the two slots is dependent (on a
  // hanging face or edge); the chains of links are the lines.  A node linked to two different nodes above (or below) makes
  // the lines inconsistent and disables the preconditioner for this mesh.
  {
    std::vector<int32_t> up((size_t)N, -1), down((size_t)N, -1);
    bool ok = true;
    std::vector<int32_t> cnt((size_t)N + 1, 0);
    for (int64_t e = 0; e < n_el && ok; ++e)
      for (int t = 0; t < P2; ++t) {
        int lo, hi;
        if (!zline_run_host(m->cmask[e], P, t % P, t / P, lo, hi)) continue;
        for (int z = lo; z <= hi; ++z) cnt[(words[e * P3 + t + P2 * z] & NODE_MASK) + 1]++;
        for (int z = lo; z < hi; ++z) {
          const int32_t a = words[e * P3 + t + P2 * z] & NODE_MASK, b = words[e * P3 + t + P2 * (z + 1)] & NODE_MASK;
          if ((up[a] != -1 && up[a] != b) || (down[b] != -1 && down[b] != a)) ok = false;
          up[a] = b;
          down[b] = a;
        }
      }
    if (ok) {
      for (int64_t n = 0; n < N; ++n) cnt[n + 1] += cnt[n];
      ctx->h_lptr.assign(cnt.begin(), cnt.end());
      ctx->h_lslot.assign(cnt[N] + 1, 0);   // + a sentinel (slot 0), so lslot[lptr[n]] is readable for every n
      std::vector<int32_t> next(cnt.begin(), cnt.end() - 1);
      for (int64_t e = 0; e < n_el; ++e)
        for (int t = 0; t < P2; ++t) {
          int lo, hi;
          if (!zline_run_host(m->cmask[e], P, t % P, t / P, lo, hi)) continue;
          for (int z = lo; z <= hi; ++z) {
            const int64_t slot = e * P3 + t + P2 * z;
            ctx->h_lslot[next[words[slot] & NODE_MASK]++] = (int32_t)slot;
          }
        }
      ctx->h_line_ptr.assign(1, 0);
      ctx->h_line_node.clear();
      ctx->h_line_node.reserve((size_t)N);
      for (int64_t n = 0; n < N; ++n) {
        if (down[n] != -1) continue;
        for (int32_t c = (int32_t)n; c != -1; c = up[c]) ctx->h_line_node.push_back(c);
        ctx->h_line_ptr.push_back((int32_t)ctx->h_line_node.size());
      }
      ok = (int64_t)ctx->h_line_node.size() == N;
    }
    ctx->lines_ok = ok;
    ctx->n_lines = ok ? (int64_t)ctx->h_line_ptr.size() - 1 : 0;
  }
  // Shared z-faces inside a block: when element e and the next element of the same block name the
  // same node at (x, y, top) and (x, y, bottom), the kernel adds the upper element's bottom value
  // to the lower element's top value and stores one entry (merged[bottom slot] = 1).
  const int64_t n_inc = n_el * P3;
  if (n_inc >= (int64_t)0x7FFFFFFF) return ctx->fail(NSMF_EUNSUP, "mesh too large for int32 entries");
  const int E = launch_elems(P);
  std::vector<uint8_t> merged((size_t)n_inc, 0);
  for (int64_t e = 0; e + 1 < n_el; ++e) {
    if (e % E == E - 1) continue;
    for (int t = 0; t < P2; ++t)
      if (words[e * P3 + P2 * (P - 1) + t] == words[(e + 1) * P3 + t]) merged[(e + 1) * P3 + t] = 1;
  }
  // node-ordered element vector: node n owns entries [iptr[n], iptr[n+1]); slot (e, a) takes
  // entry pos[e][a] = iptr[node] + (number of earlier stored slots of the same node, in element
  // order), or -1 if merged into the element below
  std::vector<int32_t> iptr((size_t)N + 1, 0), ipos((size_t)n_inc);
  for (int64_t i = 0; i < n_inc; ++i)
    if (!merged[i]) iptr[(words[i] & NODE_MASK) + 1]++;
  for (int64_t n = 0; n < N; ++n) {
    iptr[n + 1] += iptr[n];
  }
  {
    std::vector<int32_t> next(iptr.begin(), iptr.end() - 1);
    for (int64_t i = 0; i < n_inc; ++i) ipos[i] = merged[i] ? -1 : next[words[i] & NODE_MASK]++;
  }
  ctx->k = m->k;
  ctx->P = P;
  build_tables(m->k, m->pspace, &ctx->tab);
  ctx->ps = m->pspace;
  ctx->n_p = ctx->tab.n_p;
  ctx->n_el = n_el;
  ctx->n_nodes = N;
  ctx->n_bface = NB;
  ctx->nt = launch_threads(P);
  ctx->epb = launch_elems(P);
  ctx->nblocks = (int)((n_el + ctx->epb - 1) / ctx->epb);
  ctx->any_hang = any_hang;
  hipStream_t s = ctx->stream;

  NSMF_TRY(ctx, ctx->en.alloc(words.size()), "hipMalloc");
  NSMF_TRY(ctx, ctx->cmask.alloc(n_el), "hipMalloc");
  NSMF_TRY(ctx, ctx->bface_of.alloc(n_el), "hipMalloc");
  NSMF_TRY(ctx, ctx->dmask.alloc(3 * N), "hipMalloc");
  NSMF_TRY(ctx, ctx->inc_ptr.alloc(iptr.size()), "hipMalloc");
  // store order per block: the block's stored slots sorted by their entry, so that adjacent lanes
  // write adjacent entries; the LDS staging index of slot (el, x, y, z) is z E P^2 + el P^2 + x + P y,
  // with bit 15 set on a top slot that also takes the merged bottom slot of the element above
  // (P = 3, 5; P = 4 stores per thread through pos)
  const bool sorted_store = P != 4;
  const int SB = P == 5 ? store_slots<5>() : (P == 4 ? store_slots<4>() : store_slots<3>());
  std::vector<int32_t> spos(sorted_store ? (size_t)ctx->nblocks * SB : 0, -1);
  std::vector<uint16_t> sslot(sorted_store ? (size_t)ctx->nblocks * SB : 0, 0);
  if (sorted_store) {
    std::vector<std::pair<int32_t, uint16_t>> blk;
    for (int64_t lb = 0; lb < ctx->nblocks; ++lb) {
      blk.clear();
      for (int el = 0; el < E; ++el) {
        const int64_t e = lb * E + el;
        if (e >= n_el) break;
        for (int a = 0; a < P3; ++a) {
          if (ipos[e * P3 + a] < 0) continue;
          uint16_t sl = (uint16_t)((a / P2) * E * P2 + el * P2 + a % P2);
          if (a / P2 == P - 1 && el + 1 < E && e + 1 < n_el && merged[(e + 1) * P3 + a % P2]) sl |= 0x8000u;
          blk.emplace_back(ipos[e * P3 + a], sl);
        }
      }
      std::sort(blk.begin(), blk.end());
      for (size_t k = 0; k < blk.size(); ++k) {
        spos[lb * SB + k] = blk[k].first;
        sslot[lb * SB + k] = blk[k].second;
      }
    }
  }
  if (!sorted_store) NSMF_TRY(ctx, ctx->pos.alloc(ipos.size()), "hipMalloc");
  NSMF_TRY(ctx, ctx->spos.alloc(spos.size()), "hipMalloc");
  NSMF_TRY(ctx, ctx->sslot.alloc(sslot.size()), "hipMalloc");
  ctx->n_inc = n_inc;
  ctx->n_ent = iptr[N];
  NSMF_TRY(ctx, ctx->ev.alloc((size_t)3 * ctx->n_ent), "hipMalloc");
  NSMF_TRY(ctx, hipMemcpyAsync(ctx->en.p, words.data(), words.size() * 4, hipMemcpyHostToDevice, s), "copy");
  NSMF_TRY(ctx, hipMemcpyAsync(ctx->cmask.p, m->cmask, n_el * 4, hipMemcpyHostToDevice, s), "copy");
  NSMF_TRY(ctx, hipMemcpyAsync(ctx->bface_of.p, bof.data(), n_el * 4, hipMemcpyHostToDevice, s), "copy");
  NSMF_TRY(ctx, hipMemcpyAsync(ctx->dmask.p, dm.data(), 3 * N, hipMemcpyHostToDevice, s), "copy");
  if (m->n_frames > 0) {
    // per element with a framed bottom slot: the frames of its P^2 bottom slots (identity where the
    // slot's node has none), [row][9][P^2]
    std::vector<int32_t> rof((size_t)n_el, -1);
    int64_t nrow = 0;
    for (int64_t e = 0; e < n_el; ++e)
      for (int t = 0; t < P2; ++t)
        if (words[e * P3 + t] & ROT_BIT) {
          rof[e] = (int32_t)nrow++;
          break;
        }
    std::vector<double> rh((size_t)nrow * 9 * P2);
    for (int64_t e = 0; e < n_el; ++e) {
      if (rof[e] < 0) continue;
      for (int t = 0; t < P2; ++t) {
        const int32_t f = frame_row[words[e * P3 + t] & NODE_MASK];
        for (int q = 0; q < 9; ++q)
          rh[((size_t)rof[e] * 9 + q) * P2 + t] = f >= 0 ? m->frames[9 * (size_t)f + q] : (q % 4 == 0 ? 1.0 : 0.0);
      }
    }
    NSMF_TRY(ctx, ctx->rot_of.alloc(n_el), "hipMalloc");
    NSMF_TRY(ctx, ctx->rot64.alloc(rh.size()), "hipMalloc");
    NSMF_TRY(ctx, ctx->rot32.alloc(rh.size()), "hipMalloc");
    NSMF_TRY(ctx, hipMemcpyAsync(ctx->rot_of.p, rof.data(), n_el * 4, hipMemcpyHostToDevice, s), "copy");
    NSMF_TRY(ctx, hipMemcpyAsync(ctx->rot64.p, rh.data(), rh.size() * 8, hipMemcpyHostToDevice, s), "copy");
    NSMF_TRY(ctx, launch_d2f(s, ctx->rot64.p, ctx->rot32.p, (int64_t)rh.size()), "convert");
    NSMF_TRY(ctx, hipStreamSynchronize(s), "frames");
  }
  NSMF_TRY(ctx, hipMemcpyAsync(ctx->inc_ptr.p, iptr.data(), iptr.size() * 4, hipMemcpyHostToDevice, s), "copy");
  if (sorted_store) {
    NSMF_TRY(ctx, hipMemcpyAsync(ctx->spos.p, spos.data(), spos.size() * 4, hipMemcpyHostToDevice, s), "copy");
    NSMF_TRY(ctx, hipMemcpyAsync(ctx->sslot.p, sslot.data(), sslot.size() * 2, hipMemcpyHostToDevice, s), "copy");
  } else {
    NSMF_TRY(ctx, hipMemcpyAsync(ctx->pos.p, ipos.data(), ipos.size() * 4, hipMemcpyHostToDevice, s), "copy");
  }
  std::vector<double> tabset((tabset_bytes(P) + 7) / 8);
  fill_tabset(ctx->tab, tabset.data());
  NSMF_TRY(ctx, ctx->tabs.alloc(tabset.size()), "hipMalloc");
  NSMF_TRY(ctx, hipMemcpyAsync(ctx->tabs.p, tabset.data(), tabset.size() * 8, hipMemcpyHostToDevice, s), "copy");

  DevBuf<double> &X = ctx->xyz;   // kept for the low-order approximation F~
  DevBuf<unsigned> flags;
  for (int d = 0; d < 3; ++d) ctx->period[d] = m->period[d];
  NSMF_TRY(ctx, X.alloc(3 * N), "hipMalloc");
  NSMF_TRY(ctx, flags.alloc(1), "hipMalloc");
  NSMF_TRY(ctx, hipMemcpyAsync(X.p, m->coords, 3 * N * 8, hipMemcpyHostToDevice, s), "copy");
  NSMF_TRY(ctx, launch_fill(s, flags.p, 1), "fill");
  MeshView mv = ctx->mesh_view();
  NSMF_TRY(ctx, launch_geometry_impl(P, 0, s, mv, ctx->tabs.p, X.p, m->period, nullptr, nullptr, nullptr, flags.p),
           "geometry");
  unsigned hflags = 0;
  NSMF_TRY(ctx, hipMemcpyAsync(&hflags, flags.p, 4, hipMemcpyDeviceToHost, s), "copy");
  NSMF_TRY(ctx, hipStreamSynchronize(s), "geometry check");
  flags.free();
  if (hflags & 4u) {
    X.free();
    return ctx->fail(NSMF_EMESH, "inverted or degenerate element (det J <= 0 at a quadrature point)");
  }
  if (hflags & 8u) {
    X.free();
    return ctx->fail(NSMF_EMESH, "degenerate basal face");
  }
  if (hflags & 1u) {
    X.free();
    return ctx->fail(NSMF_EUNSUP, "geometry is not column-mapped (x, y must be affine in xi, eta per element)");
  }
  ctx->geo = (hflags & 2u) ? GEO_COLUMN : GEO_AFFINE;
  const size_t nqp = (size_t)ctx->nblocks * P * ctx->nt;
  const size_t nel_geo = (size_t)n_el * (ctx->geo == GEO_AFFINE ? 4 : 2);
  NSMF_TRY(ctx, ctx->geo_el64.alloc(nel_geo), "hipMalloc");
  NSMF_TRY(ctx, ctx->geo_el32.alloc(nel_geo), "hipMalloc");
  if (ctx->geo == GEO_COLUMN) {
    NSMF_TRY(ctx, ctx->geo_qp64.alloc(NGEOQP * nqp), "hipMalloc");
    NSMF_TRY(ctx, ctx->geo_qp32.alloc(NGEOQP * nqp), "hipMalloc");
    NSMF_TRY(ctx, launch_fill(s, ctx->geo_qp64.p, 2 * NGEOQP * nqp), "fill");
  }
  NSMF_TRY(ctx, ctx->face64.alloc((size_t)NB * 4 * P2), "hipMalloc");
  NSMF_TRY(ctx, ctx->face32.alloc((size_t)NB * 4 * P2), "hipMalloc");
  NSMF_TRY(ctx, launch_geometry_impl(P, ctx->geo == GEO_AFFINE ? 1 : 2, s, mv, ctx->tabs.p, X.p, m->period, ctx->geo_el64.p,
                                     ctx->geo_qp64.p, ctx->face64.p, nullptr),
           "geometry");
  NSMF_TRY(ctx, launch_d2f(s, ctx->geo_el64.p, ctx->geo_el32.p, nel_geo), "convert");
  if (ctx->geo == GEO_COLUMN) NSMF_TRY(ctx, launch_d2f(s, ctx->geo_qp64.p, ctx->geo_qp32.p, NGEOQP * nqp), "convert");
  NSMF_TRY(ctx, launch_d2f(s, ctx->face64.p, ctx->face32.p, (size_t)NB * 4 * P2), "convert");
  NSMF_TRY(ctx, hipStreamSynchronize(s), "geometry");

  // per-point state: FP64 mu', kappa, Sigma0 (8 values); FP32 mu', sqrt(kappa) Sigma0 (7 values)
  constexpr size_t NS64 = 8, NS32 = 7;
  NSMF_TRY(ctx, ctx->st64.alloc(NS64 * nqp), "hipMalloc");
  NSMF_TRY(ctx, ctx->st32.alloc(NS32 * nqp), "hipMalloc");
  NSMF_TRY(ctx, launch_fill(s, ctx->st64.p, 2 * NS64 * nqp), "fill");   // sizes in 32-bit words
  NSMF_TRY(ctx, launch_fill(s, ctx->st32.p, NS32 * nqp), "fill");
  NSMF_TRY(ctx, ctx->fst64.alloc((size_t)NB * 3 * P2), "hipMalloc");
  NSMF_TRY(ctx, ctx->fst32.alloc((size_t)NB * 3 * P2), "hipMalloc");
  NSMF_TRY(ctx, ctx->u.alloc(3 * N), "hipMalloc");
  NSMF_TRY(ctx, ctx->p.alloc((size_t)n_el * ctx->n_p), "hipMalloc");
  NSMF_TRY(ctx, ctx->logA.alloc(n_el), "hipMalloc");
  NSMF_TRY(ctx, ctx->beta64.alloc(NB > 0 ? NB : 1), "hipMalloc");
  NSMF_TRY(ctx, ctx->beta32.alloc(NB > 0 ? NB : 1), "hipMalloc");
  ctx->has_frames = m->n_frames > 0;
  ctx->have_mesh = true;
  ctx->err = "";
  return NSMF_OK;
}

int nsmf_set_params(nsmf_ctx *ctx, const nsmf_params *prm, const double *logA, const double *beta) {
  if (!ctx || !prm) return NSMF_EINVAL;
  if (!ctx->have_mesh) return ctx->fail(NSMF_ESTATE, "no mesh uploaded");
  if (!(prm->n >= 1.0) || !(prm->eps > 0.0) || !(prm->B0 > 0.0))
    return ctx->fail(NSMF_EINVAL, "need n >= 1, eps > 0, B0 > 0");
  hipStream_t s = ctx->stream;
  ctx->prm = *prm;
  if (logA)
    NSMF_TRY(ctx, hipMemcpyAsync(ctx->logA.p, logA, ctx->n_el * 8, hipMemcpyDeviceToDevice, s), "copy");
  else
    NSMF_TRY(ctx, launch_fill(s, ctx->logA.p, 2 * ctx->n_el), "fill");
  if (ctx->n_bface > 0) {
    if (beta)
      NSMF_TRY(ctx, hipMemcpyAsync(ctx->beta64.p, beta, ctx->n_bface * 8, hipMemcpyDeviceToDevice, s), "copy");
    else
      NSMF_TRY(ctx, launch_fill(s, ctx->beta64.p, 2 * ctx->n_bface), "fill");
    NSMF_TRY(ctx, launch_d2f(s, ctx->beta64.p, ctx->beta32.p, ctx->n_bface), "convert");
  }
  ctx->have_params = true;
  ctx->have_state = false;
  ctx->have_lines = false;
  ctx->have_lo = false;
  return NSMF_OK;
}

int nsmf_set_linearization(nsmf_ctx *ctx, int kind) {
  if (!ctx) return NSMF_EINVAL;
  if (kind != NSMF_NEWTON && kind != NSMF_PICARD) return ctx->fail(NSMF_EINVAL, "linearization must be 0 or 1");
  ctx->lin = kind;
  ctx->have_state = false;
  ctx->have_lines = false;
  ctx->have_lo = false;
  return NSMF_OK;
}

int nsmf_set_state(nsmf_ctx *ctx, const double *u, const double *p) {
  if (!ctx || !u || !p) return NSMF_EINVAL;
  if (!ctx->have_mesh || !ctx->have_params) return ctx->fail(NSMF_ESTATE, "set_state needs mesh and params");
  hipStream_t s = ctx->stream;
  NSMF_TRY(ctx, hipMemcpyAsync(ctx->u.p, u, 3 * ctx->n_nodes * 8, hipMemcpyDeviceToDevice, s), "copy");
  NSMF_TRY(ctx, hipMemcpyAsync(ctx->p.p, p, ctx->n_el * ctx->n_p * 8, hipMemcpyDeviceToDevice, s), "copy");
  NSMF_TRY(ctx,
           launch_state(ctx->P, ctx->geo, s, ctx->mesh_view(), ctx->geo64(), ctx->tabs.p, ctx->u.p, ctx->logA.p,
                        ctx->prm.n, ctx->prm.eps, ctx->prm.B0, ctx->lin == NSMF_PICARD, ctx->st64.p, ctx->st32.p,
                        ctx->fst64.p, ctx->fst32.p),
           "state kernel");
  ctx->have_state = true;
  ctx->have_lines = false;
  ctx->have_lo = false;
  return NSMF_OK;
}

int nsmf_residual(nsmf_ctx *ctx, const double *f_u, double *r_u, double *r_p) {
  if (!ctx || !r_u || !r_p) return NSMF_EINVAL;
  if (!ctx->have_state) return ctx->fail(NSMF_ESTATE, "residual needs a state");
  hipStream_t s = ctx->stream;
  NSMF_TRY(ctx,
           launch_residual(ctx->P, ctx->geo, ctx->ps, s, ctx->mesh_view(), ctx->geo64(), ctx->tabs.p, ctx->st64.p, ctx->fst64.p,
                           ctx->beta64.p, ctx->p.p, ctx->prm.body, ctx->ev.p, r_p),
           "residual kernel");
  NSMF_TRY(ctx, launch_assemble(s, 0, ctx->n_nodes, ctx->inc_ptr.p, ctx->ev.p, ctx->n_ent, ctx->dmask.p,
                                ctx->u.p, f_u, r_u),
           "assembly");
  return NSMF_OK;
}

static int apply_common(nsmf_ctx *ctx, int prec, bool vjp, const void *x_u, const void *x_p, void *y_u, void *y_p,
                        double *g_logA, double *g_beta) {
  if (!ctx || !x_u || !x_p) return NSMF_EINVAL;
  if (!vjp && (!y_u || !y_p)) return NSMF_EINVAL;
  if (prec < 0 || prec > 2) return ctx->fail(NSMF_EINVAL, "precision must be 0, 1 or 2");
  if (!ctx->have_state) return ctx->fail(NSMF_ESTATE, "Jacobian apply needs a state");
  if (vjp && ctx->lin != NSMF_NEWTON) return ctx->fail(NSMF_ESTATE, "residual_vjp needs the Newton linearization");
  hipStream_t s = ctx->stream;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (ctx->timing) {
    NSMF_TRY(ctx, hipEventCreate(&e0), "event");
    NSMF_TRY(ctx, hipEventCreate(&e1), "event");
    NSMF_TRY(ctx, hipEventRecord(e0, s), "event");
  }
  GeoView<double> g64 = ctx->geo64();
  GeoView<float> g32 = ctx->geo32();
  const void *gv = prec == 0 ? (const void *)&g64 : (const void *)&g32;
  // the FP32 apply reads the 7-value FP32 state; FP64 and every VJP the 8-value FP64 state
  const void *st = (prec == 0 || vjp) ? (const void *)ctx->st64.p : (const void *)ctx->st32.p;
  const void *fst = prec == 0 ? (const void *)ctx->fst64.p : (const void *)ctx->fst32.p;
  const void *beta = prec == 0 ? (const void *)ctx->beta64.p : (const void *)ctx->beta32.p;
  NSMF_TRY(ctx,
           launch_apply(ctx->P, ctx->geo, ctx->ps, prec, vjp, s, ctx->mesh_view(), gv, ctx->tabs.p, st, fst, beta, x_u, x_p,
                        y_u ? (void *)ctx->ev.p : nullptr, y_p, 1.0 / ctx->prm.n, g_logA, g_beta),
           "apply kernel");
  if (y_u)
    NSMF_TRY(ctx, launch_assemble(s, prec, ctx->n_nodes, ctx->inc_ptr.p, ctx->ev.p, ctx->n_ent, ctx->dmask.p,
                                  x_u, nullptr, y_u),
             "assembly");
  if (ctx->timing) {
    NSMF_TRY(ctx, hipEventRecord(e1, s), "event");
    ctx->events.emplace_back(e0, e1);
  }
  return NSMF_OK;
}

int nsmf_jacobian_apply(nsmf_ctx *ctx, int prec, const void *x_u, const void *x_p, void *y_u, void *y_p) {
  return apply_common(ctx, prec, false, x_u, x_p, y_u, y_p, nullptr, nullptr);
}

int nsmf_jacobian_apply_noalloc(nsmf_ctx *ctx, int prec, const void *x_u, const void *x_p, void *y_u, void *y_p) {
  if (!ctx || !x_u || !x_p || !y_u || !y_p) return NSMF_EINVAL;
  if (prec < 0 || prec > 2) return ctx->fail(NSMF_EINVAL, "precision must be 0, 1 or 2");
  if (!ctx->have_state) return ctx->fail(NSMF_ESTATE, "Jacobian apply needs a state");
  const size_t word = prec == 0 ? sizeof(double) : sizeof(float);
  const size_t need = (size_t)3 * (size_t)ctx->n_ent * word;
  if (need > NOALLOC_SCRATCH_BYTES)
    return ctx->fail(NSMF_EINVAL, "allocation-free apply: the mesh needs " + std::to_string(need) +
                                      " bytes of partial sums, the scratch array holds " +
                                      std::to_string(NOALLOC_SCRATCH_BYTES));
  if (ctx->scratch == nullptr) return ctx->fail(NSMF_EHIP, "scratch array address not resolved");
  hipStream_t s = ctx->stream;
  GeoView<double> g64 = ctx->geo64();
  GeoView<float> g32 = ctx->geo32();
  const void *gv = prec == 0 ? (const void *)&g64 : (const void *)&g32;
  const void *st = prec == 0 ? (const void *)ctx->st64.p : (const void *)ctx->st32.p;
  const void *fst = prec == 0 ? (const void *)ctx->fst64.p : (const void *)ctx->fst32.p;
  const void *beta = prec == 0 ? (const void *)ctx->beta64.p : (const void *)ctx->beta32.p;
  // every entry of the element vector is written by exactly one element slot before the assembly
  // reads it, so the scratch needs no clearing
  NSMF_TRY(ctx,
           launch_apply(ctx->P, ctx->geo, ctx->ps, prec, false, s, ctx->mesh_view(), gv, ctx->tabs.p, st, fst, beta, x_u,
                        x_p, ctx->scratch, y_p, 1.0 / ctx->prm.n, nullptr, nullptr),
           "apply kernel");
  NSMF_TRY(ctx, launch_assemble(s, prec, ctx->n_nodes, ctx->inc_ptr.p, ctx->scratch, ctx->n_ent, ctx->dmask.p, x_u,
                                nullptr, y_u),
           "assembly");
  return NSMF_OK;
}

int nsmf_gradient_apply(nsmf_ctx *ctx, int prec, const void *x_p, void *y_u) {
  if (!ctx || !x_p || !y_u) return NSMF_EINVAL;
  if (prec < 0 || prec > 2) return ctx->fail(NSMF_EINVAL, "precision must be 0, 1 or 2");
  if (!ctx->have_mesh) return ctx->fail(NSMF_ESTATE, "no mesh uploaded");
  hipStream_t s = ctx->stream;
  GeoView<double> g64 = ctx->geo64();
  GeoView<float> g32 = ctx->geo32();
  const void *gv = prec == 0 ? (const void *)&g64 : (const void *)&g32;
  NSMF_TRY(ctx, launch_grad_p(ctx->P, ctx->geo, ctx->ps, prec, s, ctx->mesh_view(), gv, ctx->tabs.p, x_p, ctx->ev.p),
           "gradient kernel");
  NSMF_TRY(ctx, launch_assemble(s, prec, ctx->n_nodes, ctx->inc_ptr.p, ctx->ev.p, ctx->n_ent, ctx->dmask.p, nullptr,
                                nullptr, y_u, 0.0),
           "assembly");
  return NSMF_OK;
}

int nsmf_residual_vjp(nsmf_ctx *ctx, int prec, const void *w_u, const void *w_p, void *g_u, void *g_p,
                      double *g_logA, double *g_beta) {
  return apply_common(ctx, prec, true, w_u, w_p, g_u, g_p, g_logA, g_beta);
}

int nsmf_lowo_apply(nsmf_ctx *ctx, const double *x_u, double *y_u) {
  if (!ctx || !x_u || !y_u) return NSMF_EINVAL;
  if (!ctx->have_state) return ctx->fail(NSMF_ESTATE, "lowo_apply needs a state");
  hipStream_t s = ctx->stream;
  if (!ctx->have_lo) {
    const size_t nlo = (size_t)NLOWO * ctx->nblocks * ctx->P * ctx->nt;
    if (ctx->lo.n != nlo) NSMF_TRY(ctx, ctx->lo.alloc(nlo), "hipMalloc");
    NSMF_TRY(ctx,
             launch_lowo_coef(ctx->P, s, ctx->mesh_view(), ctx->geo64(), ctx->tabs.p, ctx->xyz.p, ctx->period, ctx->u.p,
                              ctx->logA.p, ctx->prm.n, ctx->prm.eps, ctx->prm.B0, ctx->lin == NSMF_PICARD, ctx->lo.p),
             "low-order coefficient kernel");
    ctx->have_lo = true;
  }
  NSMF_TRY(ctx, launch_lowo(ctx->P, s, ctx->mesh_view(), ctx->geo64(), ctx->tabs.p, ctx->lo.p, ctx->beta64.p, x_u, ctx->ev.p),
           "low-order kernel");
  NSMF_TRY(ctx, launch_assemble(s, 0, ctx->n_nodes, ctx->inc_ptr.p, ctx->ev.p, ctx->n_ent, ctx->dmask.p, x_u, nullptr, y_u),
           "assembly");
  return NSMF_OK;
}

int nsmf_coarse_setup(nsmf_ctx *ctx, int64_t n_cpts, const int32_t *node_cpt, const double *node_w,
                      const double *node_zeta) {
  if (!ctx || !node_cpt || !node_w || !node_zeta) return NSMF_EINVAL;
  if (!ctx->have_mesh) return ctx->fail(NSMF_ESTATE, "no mesh uploaded");
  if (ctx->has_frames) return ctx->fail(NSMF_EUNSUP, "coarse space on a mesh with nodal frames");
  const int64_t N = ctx->n_nodes;
  if (n_cpts <= 0 || n_cpts > 0x7FFFFFFF / 16) return ctx->fail(NSMF_EINVAL, "n_cpts out of range");
  std::vector<int64_t> cnt((size_t)n_cpts + 1, 0);
  for (int64_t n = 0; n < N; ++n) {
    if (!(node_zeta[n] >= 0.0 && node_zeta[n] <= 1.0)) return ctx->fail(NSMF_EINVAL, "node_zeta outside [0, 1]");
    for (int j = 0; j < 4; ++j) {
      const int32_t J = node_cpt[4 * n + j];
      const double wv = node_w[4 * n + j];
      if (J < 0 || J >= n_cpts) return ctx->fail(NSMF_EINVAL, "node_cpt entry out of range");
      if (!std::isfinite(wv)) return ctx->fail(NSMF_EINVAL, "node_w entry not finite");
      if (wv != 0.0) cnt[J + 1]++;
    }
  }
  for (int64_t J = 0; J < n_cpts; ++J) cnt[J + 1] += cnt[J];
  std::vector<int32_t> cnode((size_t)cnt[n_cpts]);
  std::vector<double> cwt((size_t)cnt[n_cpts]);
  {
    std::vector<int64_t> next(cnt.begin(), cnt.end() - 1);
    for (int64_t n = 0; n < N; ++n)
      for (int j = 0; j < 4; ++j) {
        const double wv = node_w[4 * n + j];
        if (wv == 0.0) continue;
        const int64_t k = next[node_cpt[4 * n + j]]++;
        cnode[k] = (int32_t)n;
        cwt[k] = wv;
      }
  }
  hipStream_t s = ctx->stream;
  NSMF_TRY(ctx, ctx->c_cpt.alloc(4 * N), "hipMalloc");
  NSMF_TRY(ctx, ctx->c_w.alloc(4 * N), "hipMalloc");
  NSMF_TRY(ctx, ctx->c_zeta.alloc(N), "hipMalloc");
  NSMF_TRY(ctx, ctx->c_ptr.alloc(cnt.size()), "hipMalloc");
  NSMF_TRY(ctx, ctx->c_node.alloc(cnode.size() > 0 ? cnode.size() : 1), "hipMalloc");
  NSMF_TRY(ctx, ctx->c_wt.alloc(cwt.size() > 0 ? cwt.size() : 1), "hipMalloc");
  NSMF_TRY(ctx, hipMemcpyAsync(ctx->c_cpt.p, node_cpt, 4 * N * 4, hipMemcpyHostToDevice, s), "copy");
  NSMF_TRY(ctx, hipMemcpyAsync(ctx->c_w.p, node_w, 4 * N * 8, hipMemcpyHostToDevice, s), "copy");
  NSMF_TRY(ctx, hipMemcpyAsync(ctx->c_zeta.p, node_zeta, N * 8, hipMemcpyHostToDevice, s), "copy");
  NSMF_TRY(ctx, hipMemcpyAsync(ctx->c_ptr.p, cnt.data(), cnt.size() * 8, hipMemcpyHostToDevice, s), "copy");
  if (!cnode.empty()) {
    NSMF_TRY(ctx, hipMemcpyAsync(ctx->c_node.p, cnode.data(), cnode.size() * 4, hipMemcpyHostToDevice, s), "copy");
    NSMF_TRY(ctx, hipMemcpyAsync(ctx->c_wt.p, cwt.data(), cwt.size() * 8, hipMemcpyHostToDevice, s), "copy");
  }
  NSMF_TRY(ctx, hipStreamSynchronize(s), "coarse setup");
  ctx->n_cpts = n_cpts;
  return NSMF_OK;
}

int nsmf_coarse_prolong(nsmf_ctx *ctx, int prec, const double *xc, void *x_u) {
  if (!ctx || !xc || !x_u) return NSMF_EINVAL;
  if (prec < 0 || prec > 1) return ctx->fail(NSMF_EINVAL, "precision must be 0 or 1");
  if (ctx->n_cpts <= 0) return ctx->fail(NSMF_ESTATE, "no coarse space (nsmf_coarse_setup)");
  NSMF_TRY(ctx, launch_prolong(ctx->stream, prec, ctx->n_nodes, ctx->n_cpts, ctx->c_cpt.p, ctx->c_w.p, ctx->c_zeta.p,
                               ctx->dmask.p, xc, x_u),
           "prolongation");
  return NSMF_OK;
}

int nsmf_coarse_restrict(nsmf_ctx *ctx, int prec, const void *r_u, double *rc) {
  if (!ctx || !r_u || !rc) return NSMF_EINVAL;
  if (prec < 0 || prec > 1) return ctx->fail(NSMF_EINVAL, "precision must be 0 or 1");
  if (ctx->n_cpts <= 0) return ctx->fail(NSMF_ESTATE, "no coarse space (nsmf_coarse_setup)");
  NSMF_TRY(ctx, launch_restrict(ctx->stream, prec, ctx->n_nodes, ctx->n_cpts, ctx->c_ptr.p, ctx->c_node.p, ctx->c_wt.p,
                                ctx->c_zeta.p, ctx->dmask.p, r_u, rc),
           "restriction");
  return NSMF_OK;
}

int nsmf_jacobi_diag(nsmf_ctx *ctx, int invert, double *d_u, double *d_p) {
  if (!ctx || !d_u || !d_p) return NSMF_EINVAL;
  if (!ctx->have_state) return ctx->fail(NSMF_ESTATE, "jacobi_diag needs a state");
  hipStream_t s = ctx->stream;
  NSMF_TRY(ctx,
           launch_diag(ctx->P, ctx->geo, ctx->ps, s, ctx->mesh_view(), ctx->geo64(), ctx->tabs.p, ctx->st64.p, ctx->beta64.p,
                       ctx->ev.p, d_p),
           "diagonal kernel");
  NSMF_TRY(ctx, launch_assemble(s, 0, ctx->n_nodes, ctx->inc_ptr.p, ctx->ev.p, ctx->n_ent, ctx->dmask.p, nullptr,
                                nullptr, d_u),
           "assembly");
  if (invert) {
    NSMF_TRY(ctx, launch_recip(s, 3 * ctx->n_nodes, d_u), "reciprocal");
    NSMF_TRY(ctx, launch_recip(s, ctx->n_el * ctx->n_p, d_p), "reciprocal");
  }
  return NSMF_OK;
}

int nsmf_line_setup(nsmf_ctx *ctx, int64_t *n_lines) {
  if (!ctx) return NSMF_EINVAL;
  if (!ctx->have_state) return ctx->fail(NSMF_ESTATE, "line_setup needs a state");
  if (!ctx->lines_ok) return ctx->fail(NSMF_EUNSUP, "the mesh's vertical node lines are not consistent");
  hipStream_t s = ctx->stream;
  const int W = ctx->P;   // upper band entries per row: offsets 0..k
  if (!ctx->line_ptr.p) {
    // Interleaved line-block rows: lines in groups of LINE_GROUP, node i of line l at row
    // lrow[l] + LINE_GROUP i with lrow[l] = (group offset) + l mod LINE_GROUP, each group padded to
    // its longest line; prow[n] = row of node n.  lfirst[l] = first node of a line whose node ids are
    // consecutive, -1 otherwise.
    const int64_t NL = ctx->n_lines;
    std::vector<int32_t> prow((size_t)ctx->n_nodes), lrow((size_t)NL), lfirst((size_t)NL);
    int64_t nr = 0;
    for (int64_t g0 = 0; g0 < NL; g0 += LINE_GROUP) {
      int32_t longest = 0;
      for (int64_t l = g0; l < NL && l < g0 + LINE_GROUP; ++l)
        longest = std::max(longest, ctx->h_line_ptr[l + 1] - ctx->h_line_ptr[l]);
      for (int64_t l = g0; l < NL && l < g0 + LINE_GROUP; ++l) {
        lrow[l] = (int32_t)(nr + (l - g0));
        const int32_t b0 = ctx->h_line_ptr[l], b1 = ctx->h_line_ptr[l + 1];
        bool cons = true;
        for (int32_t q = b0; q < b1; ++q) {
          prow[ctx->h_line_node[q]] = lrow[l] + LINE_GROUP * (q - b0);
          if (q > b0) cons = cons && ctx->h_line_node[q] == ctx->h_line_node[b0] + (q - b0);
        }
        lfirst[l] = cons ? ctx->h_line_node[b0] : -1;
      }
      nr += (int64_t)LINE_GROUP * longest;
    }
    if (nr >= (int64_t)0x7FFFFFFF) return ctx->fail(NSMF_EUNSUP, "too many line-block rows for int32 indices");
    ctx->line_nr = nr;
    NSMF_TRY(ctx, ctx->line_ptr.alloc(ctx->h_line_ptr.size()), "hipMalloc");
    NSMF_TRY(ctx, ctx->line_node.alloc(ctx->h_line_node.size()), "hipMalloc");
    NSMF_TRY(ctx, ctx->line_prow.alloc(prow.size()), "hipMalloc");
    NSMF_TRY(ctx, ctx->line_row.alloc(NL > 0 ? (size_t)NL : 1), "hipMalloc");
    NSMF_TRY(ctx, ctx->line_first.alloc(NL > 0 ? (size_t)NL : 1), "hipMalloc");
    NSMF_TRY(ctx, hipMemcpyAsync(ctx->line_prow.p, prow.data(), prow.size() * 4, hipMemcpyHostToDevice, s), "copy");
    if (NL > 0) {
      NSMF_TRY(ctx, hipMemcpyAsync(ctx->line_row.p, lrow.data(), lrow.size() * 4, hipMemcpyHostToDevice, s), "copy");
      NSMF_TRY(ctx, hipMemcpyAsync(ctx->line_first.p, lfirst.data(), lfirst.size() * 4, hipMemcpyHostToDevice, s),
               "copy");
    }
    NSMF_TRY(ctx, ctx->lptr.alloc(ctx->h_lptr.size()), "hipMalloc");
    NSMF_TRY(ctx, ctx->lslot.alloc(ctx->h_lslot.size() ? ctx->h_lslot.size() : 1), "hipMalloc");
    NSMF_TRY(ctx, ctx->lbuf.alloc((size_t)3 * ctx->n_inc * W), "hipMalloc");
    NSMF_TRY(ctx, ctx->lfac64.alloc((size_t)3 * ctx->line_nr * W), "hipMalloc");
    NSMF_TRY(ctx, ctx->lfac32.alloc((size_t)3 * ctx->line_nr * W), "hipMalloc");
    NSMF_TRY(ctx, hipMemcpyAsync(ctx->line_ptr.p, ctx->h_line_ptr.data(), ctx->h_line_ptr.size() * 4,
                                 hipMemcpyHostToDevice, s), "copy");
    NSMF_TRY(ctx, hipMemcpyAsync(ctx->line_node.p, ctx->h_line_node.data(), ctx->h_line_node.size() * 4,
                                 hipMemcpyHostToDevice, s), "copy");
    NSMF_TRY(ctx, hipMemcpyAsync(ctx->lptr.p, ctx->h_lptr.data(), ctx->h_lptr.size() * 4, hipMemcpyHostToDevice, s),
             "copy");
    if (ctx->h_lslot.size())
      NSMF_TRY(ctx, hipMemcpyAsync(ctx->lslot.p, ctx->h_lslot.data(), ctx->h_lslot.size() * 4,
                                   hipMemcpyHostToDevice, s), "copy");
    NSMF_TRY(ctx, hipStreamSynchronize(s), "copy");   // the host vectors are not kept alive by the copy
  }
  NSMF_TRY(ctx,
           launch_lines(ctx->P, ctx->geo, s, ctx->mesh_view(), ctx->geo64(), ctx->tabs.p, ctx->st64.p, ctx->beta64.p,
                        ctx->lptr.p, ctx->lslot.p, ctx->dmask.p, ctx->line_ptr.p, ctx->line_node.p, ctx->line_prow.p,
                        ctx->line_row.p, ctx->line_nr, ctx->n_lines, ctx->lbuf.p, ctx->lfac64.p, ctx->lfac32.p),
           "line blocks");
  ctx->have_lines = true;
  if (n_lines) *n_lines = ctx->n_lines;
  return NSMF_OK;
}

int nsmf_line_apply(nsmf_ctx *ctx, int prec, const void *x_u, void *y_u) {
  if (!ctx || !x_u || !y_u) return NSMF_EINVAL;
  if (prec != 0 && prec != 1) return ctx->fail(NSMF_EINVAL, "line_apply precision must be 0 (double) or 1 (float)");
  if (!ctx->have_lines) return ctx->fail(NSMF_ESTATE, "line_apply needs nsmf_line_setup at the current state");
  NSMF_TRY(ctx,
           launch_line_apply(ctx->stream, prec, ctx->P, ctx->n_nodes, ctx->line_ptr.p, ctx->line_node.p,
                             ctx->line_row.p, ctx->line_nr, ctx->line_first.p, ctx->n_lines,
                             prec == 0 ? (const void *)ctx->lfac64.p : (const void *)ctx->lfac32.p, x_u, y_u),
           "line solve");
  return NSMF_OK;
}

static int vec_check(nsmf_ctx *ctx, int prec, int64_t n) {
  if (!ctx) return NSMF_EINVAL;
  if (prec != 0 && prec != 1) return ctx->fail(NSMF_EINVAL, "vector precision must be 0 (double) or 1 (float)");
  if (n <= 0) return ctx->fail(NSMF_EINVAL, "vector length must be positive");
  return NSMF_OK;
}

int nsmf_vec_dots(nsmf_ctx *ctx, int prec, int64_t n, int k, const void *V, int64_t ldv, const void *w, double *h) {
  int rc = vec_check(ctx, prec, n);
  if (rc) return rc;
  if (!V || !w || !h || k < 1 || k > MAX_DOTS || ldv < n) return ctx->fail(NSMF_EINVAL, "bad nsmf_vec_dots arguments");
  if (!ctx->dot_partial.p) NSMF_TRY(ctx, ctx->dot_partial.alloc((size_t)DOT_BLOCKS * MAX_DOTS), "hipMalloc");
  NSMF_TRY(ctx, launch_dots(ctx->stream, prec, n, k, V, ldv, w, ctx->dot_partial.p, h), "dots");
  return NSMF_OK;
}

int nsmf_vec_gemv(nsmf_ctx *ctx, int prec, int64_t n, int k, const void *V, int64_t ldv, const double *h,
                  double alpha, void *w) {
  int rc = vec_check(ctx, prec, n);
  if (rc) return rc;
  if (!V || !w || !h || k < 1 || k > MAX_DOTS || ldv < n) return ctx->fail(NSMF_EINVAL, "bad nsmf_vec_gemv arguments");
  NSMF_TRY(ctx, launch_gemv(ctx->stream, prec, n, k, V, ldv, h, alpha, w), "gemv");
  return NSMF_OK;
}

int nsmf_vec_dots_if(nsmf_ctx *ctx, const int32_t *flag, int prec, int64_t n, int k, const void *V, int64_t ldv,
                     const void *w, double *h) {
  int rc = vec_check(ctx, prec, n);
  if (rc) return rc;
  if (!flag || !V || !w || !h || k < 1 || k > MAX_DOTS || ldv < n)
    return ctx->fail(NSMF_EINVAL, "bad nsmf_vec_dots_if arguments");
  if (!ctx->dot_partial.p) NSMF_TRY(ctx, ctx->dot_partial.alloc((size_t)DOT_BLOCKS * MAX_DOTS), "hipMalloc");
  NSMF_TRY(ctx, launch_dots(ctx->stream, prec, n, k, V, ldv, w, ctx->dot_partial.p, h, flag), "dots");
  return NSMF_OK;
}

int nsmf_vec_gemv_if(nsmf_ctx *ctx, const int32_t *flag, int prec, int64_t n, int k, const void *V, int64_t ldv,
                     const double *h, double alpha, void *w) {
  int rc = vec_check(ctx, prec, n);
  if (rc) return rc;
  if (!flag || !V || !w || !h || k < 1 || k > MAX_DOTS || ldv < n)
    return ctx->fail(NSMF_EINVAL, "bad nsmf_vec_gemv_if arguments");
  NSMF_TRY(ctx, launch_gemv(ctx->stream, prec, n, k, V, ldv, h, alpha, w, flag), "gemv");
  return NSMF_OK;
}

int nsmf_gs_norm(nsmf_ctx *ctx, int k, const double *h, double eta2, const int32_t *flag_in, int32_t *flag_out,
                 double *nrm2) {
  if (!ctx) return NSMF_EINVAL;
  if (!h || !nrm2 || k < 0 || k >= MAX_DOTS || !(eta2 >= 0.0 && eta2 <= 1.0))
    return ctx->fail(NSMF_EINVAL, "bad nsmf_gs_norm arguments");
  NSMF_TRY(ctx, launch_gs_norm(ctx->stream, k, h, eta2, flag_in, flag_out, nrm2), "gs_norm");
  return NSMF_OK;
}

int nsmf_vec_axpby(nsmf_ctx *ctx, int prec, int64_t n, double a, const void *x, double b, void *y) {
  int rc = vec_check(ctx, prec, n);
  if (rc) return rc;
  if (!x || !y) return ctx->fail(NSMF_EINVAL, "NULL vector");
  NSMF_TRY(ctx, launch_axpby(ctx->stream, prec, n, a, x, b, y), "axpby");
  return NSMF_OK;
}

int nsmf_vec_normalize(nsmf_ctx *ctx, int prec, int64_t n, const double *nrm2, void *x) {
  if (!ctx || !nrm2 || !x || n < 0) return NSMF_EINVAL;
  if (prec < 0 || prec > 1) return ctx->fail(NSMF_EINVAL, "precision must be 0 or 1");
  NSMF_TRY(ctx, launch_normalize(ctx->stream, prec, n, nrm2, x), "normalize");
  return NSMF_OK;
}

int nsmf_vec_mul(nsmf_ctx *ctx, int prec, int64_t n, const double *d, const void *x, void *z) {
  int rc = vec_check(ctx, prec, n);
  if (rc) return rc;
  if (!d || !x || !z) return ctx->fail(NSMF_EINVAL, "NULL vector");
  NSMF_TRY(ctx, launch_mul(ctx->stream, prec, n, d, x, z), "mul");
  return NSMF_OK;
}

int nsmf_vec_convert(nsmf_ctx *ctx, int64_t n, int to_fp32, const void *in, void *out) {
  int rc = vec_check(ctx, 0, n);
  if (rc) return rc;
  if (!in || !out) return ctx->fail(NSMF_EINVAL, "NULL vector");
  if (to_fp32)
    NSMF_TRY(ctx, launch_d2f(ctx->stream, (const double *)in, (float *)out, n), "convert");
  else
    NSMF_TRY(ctx, launch_f2d(ctx->stream, (const float *)in, (double *)out, n), "convert");
  return NSMF_OK;
}

int nsmf_query(nsmf_ctx *ctx, int64_t *n_nodes, int64_t *n_el, int64_t *n_p, int64_t *n_dof, int64_t *n_bface) {
  if (!ctx) return NSMF_EINVAL;
  if (!ctx->have_mesh) return ctx->fail(NSMF_ESTATE, "no mesh uploaded");
  if (n_nodes) *n_nodes = ctx->n_nodes;
  if (n_el) *n_el = ctx->n_el;
  if (n_p) *n_p = ctx->n_p;
  if (n_dof) *n_dof = 3 * ctx->n_nodes + ctx->n_el * ctx->n_p;
  if (n_bface) *n_bface = ctx->n_bface;
  return NSMF_OK;
}

int nsmf_geometry_kind(nsmf_ctx *ctx) {
  if (!ctx || !ctx->have_mesh) return NSMF_ESTATE;
  return ctx->geo;
}

int nsmf_set_kernel_timing(nsmf_ctx *ctx, int enable) {
  if (!ctx) return NSMF_EINVAL;
  ctx->timing = enable != 0;
  return NSMF_OK;
}

int nsmf_kernel_time(nsmf_ctx *ctx, double *ms_total, int64_t *launches) {
  if (!ctx) return NSMF_EINVAL;
  double tot = 0.0;
  for (auto &ev : ctx->events) {
    NSMF_TRY(ctx, hipEventSynchronize(ev.second), "event");
    float ms = 0.0f;
    NSMF_TRY(ctx, hipEventElapsedTime(&ms, ev.first, ev.second), "event");
    tot += ms;
  }
  if (ms_total) *ms_total = tot;
  if (launches) *launches = (int64_t)ctx->events.size();
  for (auto &ev : ctx->events) {
    (void)hipEventDestroy(ev.first);
    (void)hipEventDestroy(ev.second);
  }
  ctx->events.clear();
  return NSMF_OK;
}

}  // extern "C"
