// C ABI of the DG MHD library: handle management, argument checking and the
// per-step launch sequence (time-step reduction, three SSP-RK3 stages, each
// face kernel -> cell kernel -> limiters), all ordered on one HIP stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <mutex>
#include <new>
#include <random>
#include <sstream>
#include <string>
#include <unordered_map>
#include <vector>

#include "../../include/dg.h"
#include "dg_kernels.h"
#include "dg_mlp.h"
#include "dg_tables.h"

using namespace dgmhd;

struct dg_handle_s {
  dg_params p{};
  Grid g{};
  SchemeParams sp{};
  Tables tabs;
  Launcher* L = nullptr;
  hipStream_t stream = nullptr;
  void* ff = nullptr;     // face fluxes
  void* jp = nullptr;     // Powell normal-field jumps
  void* S1 = nullptr;     // stage state
  void* S2 = nullptr;     // SSP-RK(5,4): two more stage states
  void* S3 = nullptr;
  void* jsum = nullptr;   // Powell per-face jump integrals
  void* lscr = nullptr;   // limiter scratch
  Scal* sc = nullptr;     // device scalars
  std::vector<void*> mesh_bufs;  // octree face lists on the device
  MlpState mlp;              // learned troubled-cell indicator
  int mlp_step = 0;          // Adam step counter
  // recording of (features, label) pairs inside dg_step
  uint16_t* rec_X = nullptr;
  float* rec_y = nullptr;
  unsigned long long* rec_counter = nullptr;
  int64_t rec_cap = 0;
  double rec_q = 0.0, rec_qpos = 1.0;
  unsigned long long rec_seed = 0;
  // one captured SSP-RK3 step per state pointer (non-null streams only)
  hipGraphExec_t graph_exec[2] = {nullptr, nullptr};  // first step of a call, later steps
  const void* graph_w = nullptr;
  std::vector<int8_t> h_level;   // octree: host copy of the leaf levels
  std::vector<int32_t> h_ijk;    // octree: host copy of the leaf coordinates
  // last regrid plan (dg_amr_plan): new leaves in Morton order, and per new
  // leaf (kind, source, depth, octant path); kids: old leaves of each merged
  // group in octant order
  std::vector<int8_t> amr_level;
  std::vector<int32_t> amr_ijk, amr_map, amr_kids;
  int64_t amr_nold = 0;
  double hmin = 0.0;
  size_t elem = 8;
  int device = 0;             // HIP device current at dg_init
  void* scratch = nullptr;    // that device's address of the file-scope scratch array
  std::string err;
};

// Workspace of dg_rhs_noalloc: the face buffer, the Powell jump buffer and
// the device scalars of one right-hand side, for callers that cannot
// allocate device memory.  One copy per device, held until the process ends;
// every dg_rhs_noalloc call on a device shares it.
static constexpr size_t kScratchBytes = (size_t)32 << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

std::string g_err;  // message for failures before a handle exists

// Device address of `scratch` per device, resolved once per device with
// that device current (the host-side name is not a device address).
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_addr[kMaxDevices] = {};

hipError_t scratch_address(int dev, void** out) {
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_addr[dev]) {
    void* p = nullptr;
    hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_addr[dev] = p;
  }
  *out = g_scratch_addr[dev];
  return hipSuccess;
}

int fail(dg_handle h, int code, const std::string& msg) {
  if (h) h->err = msg; else g_err = msg;
  return code;
}

int check_hip(dg_handle h, hipError_t e, const char* what) {
  if (e == hipSuccess) return DG_OK;
  return fail(h, DG_EHIP, std::string(what) + ": " + hipGetErrorString(e));
}

int check_launch(dg_handle h, const char* what) { return check_hip(h, hipGetLastError(), what); }

int valid_state(dg_handle h, const void* w) {
  if (!h) return DG_EINVAL;
  if (!w) return fail(h, DG_EINVAL, "null state pointer");
  return DG_OK;
}

}  // namespace

// Face lists of a periodic 2:1 octree (Sec. 4.4).  Faces are enumerated once,
// from the left cell's +a side, sorted by axis: same level (both full), a
// finer right region (one face per fine neighbour, the coarse left side on
// quarter q), or a coarser right cell (the coarse side on quarter q), q
// having bit t set when the fine face is in the upper half of the t-th
// tangential axis.  Returns an error message or "".
static std::string build_octree(dg_handle h, const dg_mesh* m) {
  const int D = h->p.dim;
  const int64_t C = m->nleaves;
  if (C <= 0 || !m->level || !m->ijk) return "octree: leaves missing";
  const int NQ = 1 << (D - 1);
  std::vector<int8_t> lev(m->level, m->level + C);
  std::vector<int32_t> ijk(m->ijk, m->ijk + 3 * C);
  int lmax = 0;
  for (int64_t c = 0; c < C; ++c) {
    if (lev[c] < 0 || lev[c] > 20) return "octree: level out of range";
    lmax = std::max(lmax, (int)lev[c]);
  }
  auto key = [](int l, int64_t i, int64_t j, int64_t k) -> uint64_t {
    return ((uint64_t)l << 60) | ((uint64_t)i << 40) | ((uint64_t)j << 20) | (uint64_t)k;
  };
  std::unordered_map<uint64_t, int32_t> idx;
  idx.reserve((size_t)C * 2);
  for (int64_t c = 0; c < C; ++c) {
    const int l = lev[c];
    for (int a = 0; a < 3; ++a) {
      const int64_t n = a < D ? ((int64_t)m->n[a] << l) : 1;
      if (ijk[3 * c + a] < 0 || ijk[3 * c + a] >= n) return "octree: coordinate outside the level grid";
    }
    if (!idx.emplace(key(l, ijk[3 * c], ijk[3 * c + 1], ijk[3 * c + 2]), (int32_t)c).second)
      return "octree: duplicate leaf";
  }
  auto find = [&](int l, int64_t* c) -> int32_t {
    if (l < 0) return -1;
    int64_t w[3] = {0, 0, 0};
    for (int a = 0; a < D; ++a) {
      const int64_t n = (int64_t)m->n[a] << l;
      w[a] = ((c[a] % n) + n) % n;
    }
    auto it = idx.find(key(l, w[0], w[1], w[2]));
    return it == idx.end() ? -1 : it->second;
  };
  std::vector<int32_t> fL, fR;
  std::vector<int8_t> sL, sR;
  int64_t face0[4] = {0, 0, 0, 0};
  for (int a = 0; a < D; ++a) {
    face0[a] = (int64_t)fL.size();
    int tang[2], nt = 0;
    for (int b = 0; b < D; ++b)
      if (b != a) tang[nt++] = b;
    for (int64_t c = 0; c < C; ++c) {
      const int l = lev[c];
      int64_t nc[3] = {ijk[3 * c], ijk[3 * c + 1], ijk[3 * c + 2]};
      nc[a] += 1;
      int32_t r = find(l, nc);
      if (r >= 0) { fL.push_back((int32_t)c); fR.push_back(r); sL.push_back(-1); sR.push_back(-1); continue; }
      int64_t pc[3] = {0, 0, 0};
      for (int b = 0; b < D; ++b) {
        const int64_t n = (int64_t)m->n[b] << l;
        pc[b] = (((nc[b] % n) + n) % n) >> 1;
      }
      r = l > 0 ? find(l - 1, pc) : -1;
      if (r >= 0) {
        int q = 0;
        for (int t = 0; t < nt; ++t) q |= (int)(ijk[3 * c + tang[t]] & 1) << t;
        fL.push_back((int32_t)c); fR.push_back(r); sL.push_back(-1); sR.push_back((int8_t)q);
        continue;
      }
      for (int q = 0; q < NQ; ++q) {
        int64_t ch[3] = {0, 0, 0};
        for (int b = 0; b < D; ++b) {
          const int64_t n = (int64_t)m->n[b] << l;
          ch[b] = 2 * (((nc[b] % n) + n) % n);
        }
        for (int t = 0; t < nt; ++t) ch[tang[t]] += (q >> t) & 1;
        r = find(l + 1, ch);
        if (r < 0) return "octree: leaves do not tile the box or are not 2:1 balanced";
        fL.push_back((int32_t)c); fR.push_back(r); sL.push_back((int8_t)q); sR.push_back(-1);
      }
    }
  }
  face0[D] = (int64_t)fL.size();
  const int64_t NF = (int64_t)fL.size();
  // side slots and coverage check
  std::vector<int32_t> slots((size_t)C * D * 2 * 4, -1);
  std::vector<int> cnt((size_t)C * D * 2, 0), full((size_t)C * D * 2, 0);
  for (int a = 0; a < D; ++a)
    for (int64_t f = face0[a]; f < face0[a + 1]; ++f) {
      const size_t kl = ((size_t)fL[f] * D + a) * 2 + 1, kr = ((size_t)fR[f] * D + a) * 2 + 0;
      if (cnt[kl] >= 4 || cnt[kr] >= 4) return "octree: too many faces on a cell side";
      slots[kl * 4 + cnt[kl]++] = (int32_t)f;
      slots[kr * 4 + cnt[kr]++] = (int32_t)f;
      full[kl] += sL[f] < 0;
      full[kr] += sR[f] < 0;
    }
  for (size_t k = 0; k < cnt.size(); ++k) {
    const bool ok = (cnt[k] == 1 && full[k] == 1) || (cnt[k] == NQ && full[k] == 0);
    if (!ok) return "octree: a cell side is not covered by one full face or 2^(D-1) quarter faces";
  }
  // face tiles for the matrix-core face kernel: per axis, the classes
  // (full, full) then (full, quarter q) then (quarter q, full), each class's
  // faces in list order, in tiles of 16 padded with -1
  std::vector<int32_t> ftile, fperm;
  {
    const int NCL = 1 + 2 * NQ;
    for (int a = 0; a < D; ++a)
      for (int k = 0; k < NCL; ++k) {
        const int wantL = k <= NQ ? -1 : k - 1 - NQ, wantR = (k >= 1 && k <= NQ) ? k - 1 : -1;
        std::vector<int32_t> list;
        for (int64_t f = face0[a]; f < face0[a + 1]; ++f)
          if (sL[f] == wantL && sR[f] == wantR) list.push_back((int32_t)f);
        for (size_t i = 0; i < list.size(); i += 16) {
          ftile.push_back(a * NCL + k);
          ftile.push_back((int32_t)fperm.size());
          for (size_t j = 0; j < 16; ++j) fperm.push_back(i + j < list.size() ? list[i + j] : -1);
        }
      }
  }
  // upload
  auto up = [&](const void* src, size_t bytes) -> void* {
    void* p = nullptr;
    if (hipMalloc(&p, bytes) != hipSuccess) return nullptr;
    h->mesh_bufs.push_back(p);
    if (hipMemcpy(p, src, bytes, hipMemcpyHostToDevice) != hipSuccess) return nullptr;
    return p;
  };
  Grid& g = h->g;
  g.level = (const int8_t*)up(lev.data(), lev.size());
  g.faceL = (const int32_t*)up(fL.data(), fL.size() * 4);
  g.faceR = (const int32_t*)up(fR.data(), fR.size() * 4);
  g.subL = (const int8_t*)up(sL.data(), sL.size());
  g.subR = (const int8_t*)up(sR.data(), sR.size());
  g.slots = (const int32_t*)up(slots.data(), slots.size() * 4);
  g.ftile = (const int32_t*)up(ftile.data(), ftile.size() * 4);
  g.fperm = (const int32_t*)up(fperm.data(), fperm.size() * 4);
  g.nftile = (int64_t)ftile.size() / 2;
  if (!g.level || !g.faceL || !g.faceR || !g.subL || !g.subR || !g.slots || !g.ftile || !g.fperm)
    return "octree: device allocation";
  g.NF = NF;
  g.ldf = (NF + 63) / 64 * 64;
  for (int a = 0; a <= 3; ++a) g.face0[a] = a <= D ? face0[a] : NF;
  g.hbase = m->box[0] / m->n[0];
  h->hmin = g.hbase / (double)(1 << lmax);
  h->h_level = lev;
  h->h_ijk = ijk;
  return "";
}

extern "C" {

int dg_init(const dg_params* p, const dg_mesh* m, void* hip_stream, dg_handle* out) {
  if (!p || !m || !out) return fail(nullptr, DG_EINVAL, "null argument");
  *out = nullptr;
  if (p->dim != 2 && p->dim != 3) return fail(nullptr, DG_EINVAL, "dim must be 2 or 3");
  if (p->degree < 1 || p->degree > 3) return fail(nullptr, DG_EUNSUPPORTED, "degree must be 1..3");
  if (p->divb != DG_GLM && p->divb != DG_POWELL) return fail(nullptr, DG_EINVAL, "unknown divb");
  if (p->precision != DG_FP64 && p->precision != DG_FP32) return fail(nullptr, DG_EINVAL, "unknown precision");
  if (p->rk_stages != 1 && p->rk_stages != 2 && p->rk_stages != 3 && p->rk_stages != 5)
    return fail(nullptr, DG_EUNSUPPORTED, "rk_stages must be 1, 2, 3 (SSP-RK of that order) or 5 (SSP-RK(5,4))");
  if (!(p->gamma > 1.0) || !(p->cfl > 0.0) || !(p->cfl < 1.0)) return fail(nullptr, DG_EINVAL, "gamma/cfl");
  if (m->kind != DG_MESH_UNIFORM && m->kind != DG_MESH_OCTREE) return fail(nullptr, DG_EINVAL, "unknown mesh kind");
  if (m->kind == DG_MESH_OCTREE) {
    if (p->divb != DG_GLM) return fail(nullptr, DG_EUNSUPPORTED, "octree meshes are built for GLM cleaning");
    if (p->limiter) return fail(nullptr, DG_EUNSUPPORTED, "limiters on octree meshes not built");
    if (!(p->glm_ch_fixed > 0.0)) return fail(nullptr, DG_EINVAL, "octree meshes need a fixed c_h (glm_ch_fixed)");
    if (m->nleaves <= 0 || !m->level || !m->ijk) return fail(nullptr, DG_EINVAL, "octree leaves missing");
  }
  if (p->powell_q != DG_POWELL_Q_MEAN && p->powell_q != DG_POWELL_Q_INTERP)
    return fail(nullptr, DG_EINVAL, "unknown powell_q");
  if (p->powell_q == DG_POWELL_Q_INTERP && p->divb != DG_POWELL)
    return fail(nullptr, DG_EINVAL, "powell_q selects the Powell scheme's q-dagger: divb must be DG_POWELL");
  if (p->limiter & ~(DG_LIM_TVB | DG_LIM_CHAR | DG_LIM_POS | DG_LIM_LEARNED))
    return fail(nullptr, DG_EINVAL, "unknown limiter flags");
  if ((p->limiter & (DG_LIM_CHAR | DG_LIM_LEARNED)) && !(p->limiter & DG_LIM_TVB))
    return fail(nullptr, DG_EINVAL, "characteristic/learned flags need DG_LIM_TVB");
  if ((p->limiter & DG_LIM_LEARNED) && (p->divb != DG_GLM || m->kind != DG_MESH_UNIFORM))
    return fail(nullptr, DG_EUNSUPPORTED, "learned indicator is built for GLM on uniform grids");
  for (int a = 0; a < p->dim; ++a)
    if (m->n[a] < 1 || !(m->box[a] > 0.0)) return fail(nullptr, DG_EINVAL, "mesh size");
  for (int a = 1; a < p->dim; ++a)
    if (std::fabs(m->box[a] / m->n[a] - m->box[0] / m->n[0]) > 1e-12 * m->box[0] / m->n[0])
      return fail(nullptr, DG_EINVAL, "cells must be cubic");
  {
    int64_t nc = 1;
    for (int a = 0; a < p->dim; ++a) nc *= m->n[a];
    if (nc > INT32_MAX) return fail(nullptr, DG_EINVAL, "more than 2^31 - 1 cells on the base grid");
  }

  dg_handle h = new (std::nothrow) dg_handle_s();
  if (!h) return fail(nullptr, DG_ENOMEM, "host allocation");
  {
    hipError_t e = hipGetDevice(&h->device);
    if (e == hipSuccess) e = scratch_address(h->device, &h->scratch);
    if (e != hipSuccess) {
      delete h;
      return fail(nullptr, DG_EHIP, std::string("scratch address: ") + hipGetErrorString(e));
    }
  }
  h->p = *p;
  h->stream = (hipStream_t)hip_stream;
  h->elem = p->precision == DG_FP64 ? 8 : 4;
  Grid& g = h->g;
  g.n0 = m->n[0];
  g.n1 = m->n[1];
  g.n2 = p->dim == 3 ? m->n[2] : 1;
  g.C = m->kind == DG_MESH_OCTREE ? m->nleaves : (int64_t)g.n0 * g.n1 * g.n2;
  g.ld = (g.C + 63) / 64 * 64;
  g.h = m->box[0] / m->n[0];
  h->hmin = g.h;
  if (m->kind == DG_MESH_OCTREE) {
    std::string e = build_octree(h, m);
    if (!e.empty()) { g_err = e; for (void* q : h->mesh_bufs) (void)hipFree(q); delete h; return DG_EINVAL; }
  }
  SchemeParams& sp = h->sp;
  sp.gamma = p->gamma;
  sp.cfl = p->cfl;
  sp.cfl_glm = p->cfl_glm > 0.0 ? p->cfl_glm : std::fmin(2.0 * p->cfl, 0.9);
  sp.glm_cr = p->glm_cr > 0.0 ? p->glm_cr : 0.18;
  sp.glm_ch_fixed = p->glm_ch_fixed;
  sp.powell_eta = p->powell_eta > 0.0 ? p->powell_eta : 0.2;
  sp.tvb_Mtilde = p->tvb_Mtilde;
  sp.tvb_beta = p->tvb_beta > 0.0 ? p->tvb_beta : 2.0;
  sp.tvb_eps = p->tvb_eps > 0.0 ? p->tvb_eps : 1e-8;
  sp.eps_rho = p->eps_rho > 0.0 ? p->eps_rho : 1e-12;
  sp.eps_p = p->eps_p > 0.0 ? p->eps_p : 1e-12;
  sp.limiter = p->limiter;
  sp.powell_q = p->powell_q;
  sp.mlp_lo = p->mlp_lo;
  sp.mlp_hi = p->mlp_hi > 0.0 ? p->mlp_hi : 0.5;
  sp.mlp_Pb = nullptr;
  sp.mlp_P = nullptr;
  sp.mlp_sigma = nullptr;

  std::string err;
  if (!build_tables(p->dim, p->degree, p->divb, h->tabs, err)) { int r = fail(nullptr, DG_EINVAL, err); delete h; return r; }
  h->L = make_launcher(p->precision, p->dim, p->degree, p->divb);
  if (!h->L) { delete h; return fail(nullptr, DG_EUNSUPPORTED, "configuration not built"); }
  auto cleanup = [&](int code, const std::string& msg) { g_err = msg; dg_destroy(h); return code; };
  hipError_t e = h->L->upload_tables(h->tabs);
  if (e != hipSuccess) return cleanup(DG_EHIP, std::string("table upload: ") + hipGetErrorString(e));
  const size_t nm = (size_t)h->L->nmodes();
  if ((e = hipMalloc(&h->ff, h->L->face_buffer_elems(g) * h->elem)) != hipSuccess) return cleanup(DG_ENOMEM, "face buffer");
  if (size_t nj = h->L->jump_buffer_elems(g, p->powell_q)) {
    if ((e = hipMalloc(&h->jp, nj * h->elem)) != hipSuccess) return cleanup(DG_ENOMEM, "jump buffer");
    if ((e = hipMalloc(&h->jsum, (size_t)2 * p->dim * g.C * sizeof(double))) != hipSuccess) return cleanup(DG_ENOMEM, "jump sums");
  }
  if ((e = hipMalloc(&h->S1, nm * g.ld * h->elem)) != hipSuccess) return cleanup(DG_ENOMEM, "stage buffer");
  if ((e = hipMemset(h->S1, 0, nm * g.ld * h->elem)) != hipSuccess) return cleanup(DG_EHIP, "stage buffer clear");
  if (p->rk_stages == 5) {
    for (void** b : {&h->S2, &h->S3}) {
      if ((e = hipMalloc(b, nm * g.ld * h->elem)) != hipSuccess) return cleanup(DG_ENOMEM, "stage buffer");
      if ((e = hipMemset(*b, 0, nm * g.ld * h->elem)) != hipSuccess) return cleanup(DG_EHIP, "stage buffer clear");
    }
  }
  if (size_t ls = h->L->limit_scratch_bytes(g)) {
    if ((e = hipMalloc(&h->lscr, ls)) != hipSuccess) return cleanup(DG_ENOMEM, "limiter scratch");
    if ((e = hipMemset(h->lscr, 0, ls)) != hipSuccess) return cleanup(DG_EHIP, "limiter scratch clear");
  }
  if ((e = hipMalloc(&h->sc, sizeof(Scal))) != hipSuccess) return cleanup(DG_ENOMEM, "scalars");
  if ((e = hipMemset(h->sc, 0, sizeof(Scal))) != hipSuccess) return cleanup(DG_EHIP, "scalars clear");
  *out = h;
  return DG_OK;
}

int dg_layout(dg_handle h, int64_t* nmodes, int64_t* ncells, int64_t* ld) {
  if (!h) return DG_EINVAL;
  if (nmodes) *nmodes = h->L->nmodes();
  if (ncells) *ncells = h->g.C;
  if (ld) *ld = h->g.ld;
  return DG_OK;
}

int dg_proj_points(dg_handle h, double* xi, int64_t* npts) {
  if (!h || !npts) return DG_EINVAL;
  *npts = h->tabs.NPROJ;
  if (xi) std::memcpy(xi, h->tabs.xproj.data(), h->tabs.xproj.size() * sizeof(double));
  return DG_OK;
}

int dg_project(dg_handle h, const double* prim, int64_t cell0, int64_t ncell, void* w) {
  if (int r = valid_state(h, w)) return r;
  if (!prim) return fail(h, DG_EINVAL, "null prim");
  if (cell0 < 0 || ncell < 0 || cell0 + ncell > h->g.C) return fail(h, DG_EINVAL, "cell range");
  if (ncell == 0) return DG_OK;
  h->L->project(prim, cell0, ncell, w, h->g, h->sp, h->stream);
  return check_launch(h, "project");
}

int dg_nodal(dg_handle h, const void* w, int64_t cell0, int64_t ncell, double* out) {
  if (int r = valid_state(h, w)) return r;
  if (!out) return fail(h, DG_EINVAL, "null out");
  if (cell0 < 0 || ncell < 0 || cell0 + ncell > h->g.C) return fail(h, DG_EINVAL, "cell range");
  if (ncell == 0) return DG_OK;
  h->L->nodal(w, cell0, ncell, out, h->g, h->stream);
  return check_launch(h, "nodal");
}

static int dt_sequence(dg_handle h, const void* w) {
  launch_reset_step(h->sc, h->stream);
  const DtFinalize fin{h->p.dim, h->p.degree, h->p.divb, h->hmin};
  const bool done = h->L->maxsig(w, h->g, h->sc, h->sp, h->stream, &fin);
  if (h->p.divb == DG_POWELL) h->L->powell_cap(w, h->jsum, h->g, h->sc, h->sp, h->stream);
  if (!done) launch_finalize_dt(h->sc, h->sp, h->p.dim, h->p.degree, h->p.divb, h->hmin, h->stream);
  return check_launch(h, "time step");
}

// Status of a completed call from its device counters: a non-finite value
// first, then the warning-class c_h check (Sec. 4.1.5: c_h is checked at
// runtime against twice the largest signal speed).
static int call_status(dg_handle h, const Scal& s) {
  if (s.nonfinite) return fail(h, DG_ENONFINITE, "non-finite value in the state");
  if (s.n_ch_violation) {
    std::ostringstream m;
    m << "fixed c_h = " << s.ch << " is below twice the largest signal speed (" << s.n_ch_violation
      << " time-step evaluation(s))";
    return fail(h, DG_ECH, m.str());
  }
  return DG_OK;
}

int dg_dt(dg_handle h, const void* w, double* dt, double* ch, double* kappa) {
  if (int r = valid_state(h, w)) return r;
  launch_reset_stats(h->sc, h->stream);
  if (int r = dt_sequence(h, w)) return r;
  Scal s;
  if (int r = check_hip(h, hipMemcpyAsync(&s, h->sc, sizeof(Scal), hipMemcpyDeviceToHost, h->stream), "copy")) return r;
  if (int r = check_hip(h, hipStreamSynchronize(h->stream), "sync")) return r;
  if (dt) *dt = s.dt;
  if (ch) *ch = s.ch;
  if (kappa) *kappa = s.kappa;
  return call_status(h, s);
}

int dg_rhs(dg_handle h, const void* w, void* dwdt, double ch, double kappa) {
  if (int r = valid_state(h, w)) return r;
  if (!dwdt || dwdt == w) return fail(h, DG_EINVAL, "dwdt must be a distinct array");
  if (h->p.divb == DG_GLM && !(ch > 0.0)) return fail(h, DG_EINVAL, "GLM needs c_h > 0");
  launch_set_scalars(h->sc, ch, kappa, 0.0, h->stream);
  h->L->face(w, h->ff, h->jp, h->g, h->sc, h->sp, h->stream);
  h->L->cell(w, w, dwdt, h->ff, h->jp, h->g, h->sc, h->sp, 0.0, 1.0, 1.0, 0, h->stream);
  return check_launch(h, "rhs");
}

int dg_rhs_noalloc(dg_handle h, const void* w, void* dwdt, double ch, double kappa) {
  if (int r = valid_state(h, w)) return r;
  if (!dwdt || dwdt == w) return fail(h, DG_EINVAL, "dwdt must be a distinct array");
  if (h->p.divb == DG_GLM && !(ch > 0.0)) return fail(h, DG_EINVAL, "GLM needs c_h > 0");
  int dev = -1;
  if (int r = check_hip(h, hipGetDevice(&dev), "get device")) return r;
  if (dev != h->device) return fail(h, DG_EINVAL, "dg_rhs_noalloc: the handle's device is not the current device");
  // layout in the scratch array: scalars, face buffer, Powell jump buffer
  const size_t off_ff = (sizeof(Scal) + 255) / 256 * 256;
  const size_t nff = h->L->face_buffer_elems(h->g) * h->elem;
  const size_t off_jp = off_ff + (nff + 255) / 256 * 256;
  const size_t need = off_jp + h->L->jump_buffer_elems(h->g, h->p.powell_q) * h->elem;
  if (need > kScratchBytes) {
    std::ostringstream m;
    m << "dg_rhs_noalloc: this mesh needs " << need << " bytes of workspace, the scratch array holds "
      << kScratchBytes;
    return fail(h, DG_EINVAL, m.str());
  }
  unsigned char* base = (unsigned char*)h->scratch;
  Scal* sc = (Scal*)base;
  void* ff = base + off_ff;
  void* jp = h->L->jump_buffer_elems(h->g, h->p.powell_q) ? (void*)(base + off_jp) : nullptr;
  launch_set_scalars(sc, ch, kappa, 0.0, h->stream);
  h->L->face(w, ff, jp, h->g, sc, h->sp, h->stream);
  h->L->cell(w, w, dwdt, ff, jp, h->g, sc, h->sp, 0.0, 1.0, 1.0, 0, h->stream);
  return check_launch(h, "rhs_noalloc");
}

int dg_limit(dg_handle h, void* w, dg_limit_stats* stats) {
  if (int r = valid_state(h, w)) return r;
  launch_reset_stats(h->sc, h->stream);
  // the characteristic GLM block needs c_h: take it from this state's time-step rule
  if ((h->p.limiter & DG_LIM_TVB) && h->p.divb == DG_GLM) {
    if (int r = dt_sequence(h, w)) return r;
  }
  if (h->rec_X)
    (void)h->L->mlp_record(w, h->rec_X, h->rec_y, h->rec_counter, h->rec_cap, h->rec_qpos, h->rec_q, h->rec_seed,
                           h->g, h->sc, h->sp, h->stream);
  if (h->p.limiter) h->L->limit(w, h->lscr, h->g, h->sc, h->sp, h->stream);
  if (int r = check_launch(h, "limit")) return r;
  if (stats) {
    launch_scan_nonfinite(w, h->elem, h->L->nmodes(), h->g.ld, h->g.C, h->sc, h->stream);
    if (int r = check_launch(h, "scan")) return r;
    Scal s;
    if (int r = check_hip(h, hipMemcpyAsync(&s, h->sc, sizeof(Scal), hipMemcpyDeviceToHost, h->stream), "copy")) return r;
    if (int r = check_hip(h, hipStreamSynchronize(h->stream), "sync")) return r;
    stats->n_tvb_triggered = (int64_t)s.n_tvb;
    stats->n_mlp_flagged = (int64_t)s.n_mlp;
    stats->n_fallback = (int64_t)s.n_fallback;
    stats->n_pos_scaled = (int64_t)s.n_pos;
    stats->n_floor = (int64_t)s.n_floor;
    stats->n_ch_violation = (int64_t)s.n_ch_violation;
    stats->injected_mass = s.inj_mass;
    stats->injected_energy = s.inj_energy;
    stats->max_signal = s.last_maxsig;
    stats->ch = s.ch;
    return call_status(h, s);
  }
  return DG_OK;
}

// The launch sequence of one SSP-RK3 step: device time-step reduction, then
// per stage the face kernel, the cell kernel (stage combination fused) and
// the limiters.  Kernels only: the sequence can be captured into a graph.
// first: the first step of a dg_step call.  Where the positivity limiter can
// fold the max signal speed of its output into the next step's slots
// (fused_signal), later steps take their time-step reduction from there
// instead of evaluating the state again.
static void step_sequence(dg_handle h, void* w, bool first) {
  const bool lim = h->p.limiter != 0;
  const bool fused = lim && h->L->fused_signal(h->g, h->sp);
  // Powell (normal-field jumps in jp): the first stage's face kernel runs
  // before the time step, whose cap then reads the jumps it wrote
  bool face_ready = false;
  // where the reduction finalises the step itself it also leaves its maxima
  // clear, so only the first step of a call resets them
  const bool self_final = h->p.divb == DG_GLM && h->L->maxsig_finalizes(h->g);
  bool finalized = false;
  if (first || !fused) {
    if (first || !self_final) launch_reset_step(h->sc, h->stream);
    const DtFinalize fin{h->p.dim, h->p.degree, h->p.divb, h->hmin};
    finalized = h->L->maxsig(w, h->g, h->sc, h->sp, h->stream, &fin);
    if (h->p.divb == DG_POWELL) {
      if (!h->sp.powell_q && !h->g.level) {
        h->L->face(w, h->ff, h->jp, h->g, h->sc, h->sp, h->stream);
        h->L->powell_cap_jp(w, h->jp, h->jsum, h->g, h->sc, h->stream);
        face_ready = true;
      } else {
        h->L->powell_cap(w, h->jsum, h->g, h->sc, h->sp, h->stream);
      }
    }
  } else {
    launch_take_next(h->sc, h->stream);
  }
  if (!finalized) launch_finalize_dt(h->sc, h->sp, h->p.dim, h->p.degree, h->p.divb, h->hmin, h->stream);
  auto record = [&](void* u) {
    if (h->rec_X)
      (void)h->L->mlp_record(u, h->rec_X, h->rec_y, h->rec_counter, h->rec_cap, h->rec_qpos, h->rec_q, h->rec_seed,
                             h->g, h->sc, h->sp, h->stream);
  };
  // one Shu-Osher stage: out = a0 base + b0 (in + c0 dt L(in)), then the
  // limiters (the last stage of the step also folds the next step's signal)
  auto stage = [&](void* in, void* base, void* out, double a0, double b0, double c0, bool last) {
    // the stages' face launches feed no Powell cap (the step's cap, if any,
    // comes from the launch ahead of the time step)
    if (!(face_ready && in == w)) h->L->face(in, h->ff, h->jp, h->g, h->sc, h->sp, h->stream, false);
    face_ready = false;
    h->L->cell(in, base, out, h->ff, h->jp, h->g, h->sc, h->sp, a0, b0, c0, 1, h->stream);
    record(out);
    if (last && fused) launch_reset_next(h->sc, h->stream);
    if (lim) h->L->limit(out, h->lscr, h->g, h->sc, h->sp, h->stream, last && fused);
  };
  switch (h->p.rk_stages) {
    case 1:  // forward Euler: w = w + dt L(w)
      stage(w, w, w, 0.0, 1.0, 1.0, true);
      break;
    case 2:  // SSP-RK2: S1 = w + dt L(w); w = w/2 + (S1 + dt L(S1))/2
      stage(w, w, h->S1, 0.0, 1.0, 1.0, false);
      stage(h->S1, w, w, 0.5, 0.5, 1.0, true);
      break;
    case 5: {
      // SSP-RK(5,4) in Shu-Osher form (coefficients of the five-stage,
      // fourth-order SSP scheme):
      //   u1 = u0 + b10 dt L0;   u2 = a20 u0 + a21 u1 + b21 dt L1;
      //   u3 = a30 u0 + a32 u2 + b32 dt L2;   u4 = a40 u0 + a43 u3 + b43 dt L3;
      //   u5 = a52 u2 + a53 u3 + b53 dt L3 + a54 u4 + b54 dt L4.
      // Buffers: u1 -> S1, u2 -> S2, u3 -> S1, u4 -> S3.  Before u4 is
      // limited, Q = a52 u2 + a53 u3 + b53 dt L3 is formed into S2 with
      // dt L3 = (u4 - a40 u0 - a43 u3) / b43; then u5 = Q + a54 (u4 + b54/a54 dt L4).
      const double b10 = 0.391752226571890;
      const double a20 = 0.444370493651235, a21 = 0.555629506348765, b21 = 0.368410593050371;
      const double a30 = 0.620101851488403, a32 = 0.379898148511597, b32 = 0.251891774271694;
      const double a40 = 0.178079954393132, a43 = 0.821920045606868, b43 = 0.544974750228521;
      const double a52 = 0.517231671970585, a53 = 0.096059710526147, b53 = 0.063692468666290;
      const double a54 = 0.386708617503269, b54 = 0.226007483236906;
      stage(w, w, h->S1, 0.0, 1.0, b10, false);
      stage(h->S1, w, h->S2, a20, a21, b21 / a21, false);
      stage(h->S2, w, h->S1, a30, a32, b32 / a32, false);
      // u4 unlimited, then Q, then the limiters on u4
      h->L->face(h->S1, h->ff, h->jp, h->g, h->sc, h->sp, h->stream, false);
      h->L->cell(h->S1, w, h->S3, h->ff, h->jp, h->g, h->sc, h->sp, a40, a43, b43 / a43, 1, h->stream);
      {
        const double k = b53 / b43;
        const void* x[4] = {w, h->S1, h->S2, h->S3};
        const double c[4] = {-k * a40, a53 - k * a43, a52, k};
        launch_lincomb(h->S2, x, c, h->elem, h->L->nmodes(), h->g.ld, h->g.C, h->stream);
      }
      record(h->S3);
      if (lim) h->L->limit(h->S3, h->lscr, h->g, h->sc, h->sp, h->stream);
      stage(h->S3, h->S2, w, 1.0, a54, b54 / a54, true);
      break;
    }
    default:  // SSP-RK3 (Shu-Osher)
      stage(w, w, h->S1, 0.0, 1.0, 1.0, false);                     // S1 = w + dt L(w)
      stage(h->S1, w, h->S1, 0.75, 0.25, 1.0, false);               // S1 = 3/4 w + 1/4 (S1 + dt L(S1))
      stage(h->S1, w, w, 1.0 / 3.0, 2.0 / 3.0, 1.0, true);          // w = 1/3 w + 2/3 (S1 + dt L(S1))
      break;
  }
}

static void drop_graph(dg_handle h) {
  for (int k = 0; k < 2; ++k) {
    if (h->graph_exec[k]) (void)hipGraphExecDestroy(h->graph_exec[k]);
    h->graph_exec[k] = nullptr;
  }
  h->graph_w = nullptr;
}

// Capture the first and the later steps for state w on the handle's
// (non-null) stream.
static int capture_step(dg_handle h, void* w) {
  drop_graph(h);
  for (int k = 0; k < 2; ++k) {
    hipGraph_t graph = nullptr;
    if (int r = check_hip(h, hipStreamBeginCapture(h->stream, hipStreamCaptureModeThreadLocal), "begin capture"))
      return r;
    step_sequence(h, w, k == 0);
    hipError_t e = hipStreamEndCapture(h->stream, &graph);
    if (e != hipSuccess) return check_hip(h, e, "end capture");
    e = hipGraphInstantiate(&h->graph_exec[k], graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess) {
      h->graph_exec[k] = nullptr;
      drop_graph(h);
      return check_hip(h, e, "graph instantiate");
    }
  }
  h->graph_w = w;
  return DG_OK;
}

int dg_step(dg_handle h, void* w, int32_t nsteps, double* t) {
  if (int r = valid_state(h, w)) return r;
  if (nsteps < 0) return fail(h, DG_EINVAL, "nsteps < 0");
  launch_set_time(h->sc, 0.0, h->stream);  // device clock of this call
  launch_reset_stats(h->sc, h->stream);
  const bool graph = h->stream != nullptr && nsteps > 0;
  if (graph && (h->graph_w != w || !h->graph_exec[0] || !h->graph_exec[1])) {
    if (int r = capture_step(h, w)) return r;
  }
  for (int32_t n = 0; n < nsteps; ++n) {
    if (graph) {
      if (int r = check_hip(h, hipGraphLaunch(h->graph_exec[n == 0 ? 0 : 1], h->stream), "graph launch")) return r;
    } else {
      step_sequence(h, w, n == 0);
      if (int r = check_launch(h, "step")) return r;
    }
  }
  if (t) {
    launch_scan_nonfinite(w, h->elem, h->L->nmodes(), h->g.ld, h->g.C, h->sc, h->stream);
    if (int r = check_launch(h, "scan")) return r;
    Scal s;
    if (int r = check_hip(h, hipMemcpyAsync(&s, h->sc, sizeof(Scal), hipMemcpyDeviceToHost, h->stream), "copy")) return r;
    if (int r = check_hip(h, hipStreamSynchronize(h->stream), "sync")) return r;
    *t += s.t;
    return call_status(h, s);
  }
  return DG_OK;
}


int dg_time_kernel(dg_handle h, const void* w, int32_t which, int32_t reps, double* ms) {
  if (int r = valid_state(h, w)) return r;
  if (!ms || reps < 1 || which < 0 || which > 3) return fail(h, DG_EINVAL, "time_kernel arguments");
  // workspaces: the face buffer is filled once so the cell kernel reads valid fluxes
  if (int r = dt_sequence(h, w)) return r;
  h->L->face(w, h->ff, h->jp, h->g, h->sc, h->sp, h->stream);
  if (which == 3) {
    const size_t bytes = (size_t)h->L->nmodes() * h->g.ld * h->elem;
    if (int r = check_hip(h, hipMemcpyAsync(h->S1, w, bytes, hipMemcpyDeviceToDevice, h->stream), "copy")) return r;
  }
  hipEvent_t e0, e1;
  if (int r = check_hip(h, hipEventCreate(&e0), "event")) return r;
  if (int r = check_hip(h, hipEventCreate(&e1), "event")) { (void)hipEventDestroy(e0); return r; }
  (void)hipEventRecord(e0, h->stream);
  for (int i = 0; i < reps; ++i) {
    switch (which) {
      case 0: h->L->face(w, h->ff, h->jp, h->g, h->sc, h->sp, h->stream); break;
      case 1:
        // the step's mix: one stage-1 form (w -> S1) per two stage-2/3 forms
        // (S1 and w read, S1 written in place); w is only read
        if (i % 3 == 0) h->L->cell(w, w, h->S1, h->ff, h->jp, h->g, h->sc, h->sp, 0.0, 1.0, 1.0, 1, h->stream);
        else h->L->cell(h->S1, w, h->S1, h->ff, h->jp, h->g, h->sc, h->sp, 0.75, 0.25, 1.0, 1, h->stream);
        break;
      case 2: (void)dt_sequence(h, w); break;
      default: h->L->limit(h->S1, h->lscr, h->g, h->sc, h->sp, h->stream); break;
    }
  }
  (void)hipEventRecord(e1, h->stream);
  int rc = check_hip(h, hipEventSynchronize(e1), "event sync");
  float t = 0.f;
  if (rc == DG_OK) rc = check_hip(h, hipEventElapsedTime(&t, e0, e1), "elapsed");
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (rc == DG_OK) rc = check_launch(h, "time_kernel");
  *ms = (double)t / reps;
  return rc;
}

// Cache key of a schedule: precision, dimension, degree, scheme, Powell q,
// cell count and, on octrees, the level mix (leaves per level) and the share
// of faces between levels, which set the cost of the sub-face gathers.
static std::string tune_key(dg_handle h) {
  std::ostringstream k;
  k << "sched/p" << h->p.precision << "/D" << h->p.dim << "/d" << h->p.degree << "/b" << h->p.divb << "/q"
    << h->p.powell_q << "/C" << h->g.C;
  if (!h->h_level.empty()) {
    int64_t cnt[21] = {0};
    for (int8_t l : h->h_level) cnt[l >= 0 && l <= 20 ? l : 0] += 1;
    k << "/L";
    for (int l = 0; l <= 20; ++l)
      if (cnt[l]) k << l << ":" << cnt[l] << ",";
    k << "/F" << h->g.NF;
  }
  return k.str();
}

// Minimal JSON object of "key": integer pairs, one per line.
static bool tune_cache_lookup(const char* path, const std::string& key, int& v) {
  std::ifstream f(path);
  if (!f) return false;
  std::string line, want = "\"" + key + "\"";
  while (std::getline(f, line)) {
    size_t p = line.find(want);
    if (p == std::string::npos) continue;
    size_t c = line.find(':', p + want.size());
    if (c == std::string::npos) continue;
    v = std::atoi(line.c_str() + c + 1);
    return true;
  }
  return false;
}

static void tune_cache_store(const char* path, const std::string& key, int v, double ms) {
  std::vector<std::string> entries;
  {
    std::ifstream f(path);
    std::string line;
    while (f && std::getline(f, line)) {
      size_t q = line.find('"');
      if (q == std::string::npos || line.find(':') == std::string::npos) continue;
      if (line.find("\"" + key + "\"") != std::string::npos) continue;
      std::string e = line.substr(q);
      while (!e.empty() && (e.back() == ',' || e.back() == ' ' || e.back() == '\r')) e.pop_back();
      entries.push_back(e);
    }
  }
  std::ostringstream e;
  e << "\"" << key << "\": " << v;
  entries.push_back(e.str());
  std::ofstream o(path, std::ios::trunc);
  o << "{\n";
  for (size_t i = 0; i < entries.size(); ++i) o << "  " << entries[i] << (i + 1 < entries.size() ? ",\n" : "\n");
  o << "}\n";
  (void)ms;
}

// A schedule is (cell variant) + 16 x (face variant); the two kernels must
// agree on the face-flux layout (points or moments) of the grid.
static bool schedule_valid(Launcher* L, const Grid& g, int v) {
  const int cv = v & 15, fv = v >> 4;
  return v >= 0 && cv < L->cell_variant_count() && L->cell_variant_valid(cv) && fv < L->face_variant_count() &&
         L->layout_compatible(cv, fv, g);
}

static void set_schedule(dg_handle h, int v) {
  h->L->set_cell_variant(v & 15);
  h->L->set_face_variant(v >> 4);
  drop_graph(h);
}

int dg_autotune(dg_handle h, const void* w, const char* cache_path, int32_t* variant) {
  if (int r = valid_state(h, w)) return r;
  if (!variant) return fail(h, DG_EINVAL, "null variant");
  Launcher* L = h->L;
  if (*variant >= 0) {
    if (!schedule_valid(L, h->g, *variant))
      return fail(h, DG_EINVAL, "kernel variant not built for this configuration, or cell and face kernels that exchange different face-flux layouts");
    set_schedule(h, *variant);
    return DG_OK;
  }
  const std::string key = tune_key(h);
  int cached = -1;
  if (cache_path && tune_cache_lookup(cache_path, key, cached) && schedule_valid(L, h->g, cached)) {
    set_schedule(h, cached);
    *variant = cached;
    return DG_OK;
  }
  // the cell and face kernels are timed on their own (each reads only its
  // inputs), then the fastest compatible pair is kept
  std::vector<double> cms(L->cell_variant_count(), 1e300), fms(L->face_variant_count(), 1e300);
  for (int v = 0; v < L->cell_variant_count(); ++v) {
    if (!L->cell_variant_valid(v)) continue;
    L->set_cell_variant(v);
    double ms = 0.0;
    if (int r = dg_time_kernel(h, w, 1, 1, &ms)) return r;  // warm-up
    if (int r = dg_time_kernel(h, w, 1, 3, &ms)) return r;
    cms[v] = ms;
  }
  for (int v = 0; v < L->face_variant_count(); ++v) {
    L->set_face_variant(v);
    double ms = 0.0;
    if (int r = dg_time_kernel(h, w, 0, 1, &ms)) return r;
    if (int r = dg_time_kernel(h, w, 0, 3, &ms)) return r;
    fms[v] = ms;
  }
  int best = -1;
  double best_ms = 1e300;
  for (int c = 0; c < L->cell_variant_count(); ++c)
    for (int f = 0; f < L->face_variant_count(); ++f)
      if (schedule_valid(L, h->g, c + 16 * f) && cms[c] + fms[f] < best_ms) {
        best_ms = cms[c] + fms[f];
        best = c + 16 * f;
      }
  if (best < 0) return fail(h, DG_EUNSUPPORTED, "no cell variant built");
  set_schedule(h, best);
  *variant = best;
  if (cache_path) tune_cache_store(cache_path, key, best, best_ms);
  return DG_OK;
}

static int mlp_ready(dg_handle h) {
  if (h->p.divb != DG_GLM || h->g.level) return fail(h, DG_EUNSUPPORTED, "learned indicator: GLM on uniform grids");
  std::string e;
  if (!h->mlp.alloc_params(e)) return fail(h, DG_ENOMEM, e);
  return DG_OK;
}

int dg_mlp_scale(dg_handle h, const void* w, double* sigma) {
  if (int r = valid_state(h, w)) return r;
  if (int r = mlp_ready(h)) return r;
  double* part = nullptr;
  const int64_t nblk = (h->g.C + 255) / 256;
  if (int r = check_hip(h, hipMalloc(&part, (size_t)nblk * 9 * sizeof(double)), "scale buffer")) return r;
  if (!h->L->mlp_scale(w, part, h->mlp.sigma, h->g, h->stream)) { (void)hipFree(part); return fail(h, DG_EUNSUPPORTED, "scale"); }
  int rc = check_hip(h, hipStreamSynchronize(h->stream), "sync");
  (void)hipFree(part);
  if (rc) return rc;
  h->mlp.have_sigma = true;
  if (sigma) rc = check_hip(h, hipMemcpy(sigma, h->mlp.sigma, 9 * sizeof(double), hipMemcpyDeviceToHost), "sigma");
  return rc;
}

int dg_mlp_set(dg_handle h, const float* params, const double* sigma, uint64_t seed) {
  if (!h) return DG_EINVAL;
  if (int r = mlp_ready(h)) return r;
  if (!sigma && !h->mlp.have_sigma) return fail(h, DG_EINVAL, "no feature scales: pass sigma or call dg_mlp_scale");
  std::vector<float> pub(MLP_NPARAM, 0.f), dev;
  if (params) {
    std::memcpy(pub.data(), params, sizeof(float) * MLP_NPARAM);
  } else {
    // W ~ U(-1/sqrt(fin), 1/sqrt(fin)), b = 0
    std::mt19937_64 rng(seed);
    std::uniform_real_distribution<double> U(-1.0, 1.0);
    const int fin[4] = {256, 64, 64, 64}, fo[4] = {64, 64, 64, 1};
    size_t q = 0;
    for (int l = 0; l < 4; ++l) {
      const double lim = 1.0 / std::sqrt((double)fin[l]);
      for (int i = 0; i < fin[l] * fo[l]; ++i) pub[q++] = (float)(lim * U(rng));
      q += fo[l];
    }
  }
  mlp_pack(pub.data(), dev);
  MlpState& M = h->mlp;
  if (int r = check_hip(h, hipMemcpy(M.P, dev.data(), dev.size() * 4, hipMemcpyHostToDevice), "mlp upload")) return r;
  if (int r = check_hip(h, hipMemset(M.Mo, 0, dev.size() * 4), "mlp adam")) return r;
  if (int r = check_hip(h, hipMemset(M.Vo, 0, dev.size() * 4), "mlp adam")) return r;
  if (sigma) {
    if (int r = check_hip(h, hipMemcpy(M.sigma, sigma, 9 * sizeof(double), hipMemcpyHostToDevice), "sigma")) return r;
    M.have_sigma = true;
  }
  M.sync_bf16(h->stream);
  if (int r = check_hip(h, hipStreamSynchronize(h->stream), "sync")) return r;
  h->mlp_step = 0;
  h->sp.mlp_Pb = M.Pb;
  h->sp.mlp_P = M.P;
  h->sp.mlp_sigma = M.sigma;
  M.have_params = true;
  drop_graph(h);
  return DG_OK;
}

int dg_mlp_get(dg_handle h, float* params) {
  if (!h || !params) return DG_EINVAL;
  if (!h->mlp.have_params) return fail(h, DG_EINVAL, "no network installed");
  std::vector<float> dev(MLP_NPARAM_DEV);
  if (int r = check_hip(h, hipStreamSynchronize(h->stream), "sync")) return r;
  if (int r = check_hip(h, hipMemcpy(dev.data(), h->mlp.P, dev.size() * 4, hipMemcpyDeviceToHost), "download")) return r;
  mlp_unpack(dev, params);
  return DG_OK;
}

int dg_mlp_features(dg_handle h, const void* w, void* X) {
  if (int r = valid_state(h, w)) return r;
  if (!X) return fail(h, DG_EINVAL, "null X");
  if (!h->mlp.have_params) return fail(h, DG_EINVAL, "dg_mlp_set first (feature scales)");
  if (!h->L->mlp_features(w, (uint16_t*)X, h->mlp.sigma, h->g, h->stream)) return fail(h, DG_EUNSUPPORTED, "features");
  return check_launch(h, "features");
}

int dg_mlp_labels(dg_handle h, const void* w, float* y) {
  if (int r = valid_state(h, w)) return r;
  if (!y) return fail(h, DG_EINVAL, "null y");
  if (int r = dt_sequence(h, w)) return r;  // c_h of this state for the GLM block
  if (!h->L->mlp_labels(w, y, h->g, h->sc, h->sp, h->stream)) return fail(h, DG_EUNSUPPORTED, "labels");
  return check_launch(h, "labels");
}

int dg_mlp_record(dg_handle h, void* X, float* y, unsigned long long* counter, int64_t cap, double q_pos,
                  double q_neg, uint64_t seed) {
  if (!h) return DG_EINVAL;
  if (X && (!y || !counter || cap <= 0)) return fail(h, DG_EINVAL, "record buffers");
  if (X && !h->mlp.have_params) return fail(h, DG_EINVAL, "dg_mlp_set first (feature scales)");
  h->rec_X = (uint16_t*)X;
  h->rec_y = y;
  h->rec_counter = counter;
  h->rec_cap = cap;
  h->rec_q = q_neg;
  h->rec_qpos = q_pos;
  h->rec_seed = seed;
  drop_graph(h);
  return DG_OK;
}

int dg_mlp_forward(dg_handle h, const void* X, int64_t nrows, float* prob) {
  if (!h || !X || !prob || nrows < 0) return DG_EINVAL;
  if (!h->mlp.have_params) return fail(h, DG_EINVAL, "no network installed");
  std::string e;
  MlpState& M = h->mlp;
  if (!M.alloc(M.B > 0 ? M.B : 4096, e)) return fail(h, DG_ENOMEM, e);
  for (int64_t r0 = 0; r0 < nrows; r0 += M.B) {
    const int64_t nr = std::min<int64_t>(M.B, nrows - r0);
    M.gather((const uint16_t*)X, nullptr, nullptr, r0, nrows, h->stream);
    M.forward(h->stream);
    mlp_head_probs(M, h->stream);
    if (int r = check_hip(h, hipMemcpyAsync(prob + r0, M.pout, nr * 4, hipMemcpyDeviceToDevice, h->stream), "copy"))
      return r;
  }
  return check_launch(h, "mlp forward");
}

int dg_mlp_grad(dg_handle h, const void* X, const float* y, int64_t nrows, float* grads, float* loss) {
  if (!h || !X || !y || !grads || nrows <= 0) return DG_EINVAL;
  if (!h->mlp.have_params) return fail(h, DG_EINVAL, "no network installed");
  std::string e;
  MlpState& M = h->mlp;
  if (!M.alloc((int)nrows, e)) return fail(h, DG_ENOMEM, e);
  mlp_zero_loss(M, 0, h->stream);
  M.loss_slot = 0;
  M.gather((const uint16_t*)X, y, nullptr, 0, nrows, h->stream);
  M.backward(nrows, h->stream);
  std::vector<float> dev(MLP_NPARAM_DEV);
  float l = 0.f;
  if (int r = check_hip(h, hipStreamSynchronize(h->stream), "sync")) return r;
  if (int r = check_hip(h, hipMemcpy(dev.data(), M.G, dev.size() * 4, hipMemcpyDeviceToHost), "download")) return r;
  if (int r = check_hip(h, hipMemcpy(&l, M.loss, 4, hipMemcpyDeviceToHost), "download")) return r;
  mlp_unpack(dev, grads);
  if (loss) *loss = l;
  return DG_OK;
}

int dg_mlp_train(dg_handle h, const void* X, const float* y, int64_t nrows, int32_t batch, int32_t epochs, float lr,
                 uint64_t seed, float* losses) {
  if (!h || !X || !y || nrows <= 0 || batch < 16 || epochs < 1 || epochs > 4096 || !(lr > 0.f)) return DG_EINVAL;
  if (!h->mlp.have_params) return fail(h, DG_EINVAL, "no network installed");
  std::string e;
  MlpState& M = h->mlp;
  if (!M.alloc(batch, e)) return fail(h, DG_ENOMEM, e);
  int32_t* idx = nullptr;
  if (int r = check_hip(h, hipMalloc(&idx, (size_t)nrows * 4), "index")) return r;
  std::vector<int32_t> perm((size_t)nrows);
  std::mt19937_64 rng(seed);
  int rc = DG_OK;
  for (int ep = 0; ep < epochs && rc == DG_OK; ++ep) {
    for (int64_t i = 0; i < nrows; ++i) perm[i] = (int32_t)i;
    for (int64_t i = nrows - 1; i > 0; --i) std::swap(perm[i], perm[std::uniform_int_distribution<int64_t>(0, i)(rng)]);
    rc = check_hip(h, hipMemcpyAsync(idx, perm.data(), (size_t)nrows * 4, hipMemcpyHostToDevice, h->stream), "idx");
    if (rc) break;
    mlp_zero_loss(M, ep, h->stream);
    M.loss_slot = ep;
    int64_t nb_ = 0;
    for (int64_t r0 = 0; r0 + M.B <= nrows; r0 += M.B, ++nb_) {  // full batches only
      M.gather((const uint16_t*)X, y, idx, r0, nrows, h->stream);
      M.backward(M.B, h->stream);
      M.adam(lr, ++h->mlp_step, h->stream);
    }
    rc = check_hip(h, hipStreamSynchronize(h->stream), "epoch");  // the host permutation buffer is reused
    if (rc == DG_OK && losses) {
      float l = 0.f;
      rc = check_hip(h, hipMemcpy(&l, M.loss + ep, 4, hipMemcpyDeviceToHost), "loss");
      losses[ep] = nb_ ? l / (float)nb_ : 0.f;
    }
  }
  (void)hipFree(idx);
  drop_graph(h);
  if (rc) return rc;
  return check_launch(h, "mlp train");
}

const char* dg_last_error(dg_handle h) { return h ? h->err.c_str() : g_err.c_str(); }

// ---------------------------------------------------------------------------
// Dynamic refinement (Sec. 4.4)

namespace {

using LeafKey = uint64_t;
inline LeafKey leaf_key(int l, int64_t i, int64_t j, int64_t k) {
  return ((uint64_t)l << 60) | ((uint64_t)i << 40) | ((uint64_t)j << 20) | (uint64_t)k;
}

struct LeafSet {
  int D = 3;
  int64_t n0[3] = {1, 1, 1};
  std::vector<int8_t> lev;
  std::vector<int32_t> ijk;  // [C][3]
  std::unordered_map<LeafKey, int64_t> index;
  void build_index() {
    index.clear();
    index.reserve(lev.size() * 2);
    for (size_t c = 0; c < lev.size(); ++c) index.emplace(leaf_key(lev[c], ijk[3 * c], ijk[3 * c + 1], ijk[3 * c + 2]), (int64_t)c);
  }
  int64_t ncell(int l, int a) const { return a < D ? (n0[a] << l) : 1; }
  bool is_leaf(int l, const int64_t* c) const {
    if (l < 0) return false;
    int64_t w[3] = {0, 0, 0};
    for (int a = 0; a < D; ++a) {
      const int64_t n = ncell(l, a);
      w[a] = ((c[a] % n) + n) % n;
    }
    return index.count(leaf_key(l, w[0], w[1], w[2])) > 0;
  }
  // leaves with a face neighbour more than one level finer (2:1 rule)
  std::vector<char> balance_violations() const {
    const int64_t C = (int64_t)lev.size();
    std::vector<char> bad((size_t)C, 0);
    for (int64_t i = 0; i < C; ++i) {
      const int l = lev[i];
      for (int a = 0; a < D; ++a)
        for (int sg = -1; sg <= 1; sg += 2) {
          int64_t nc[3] = {ijk[3 * i], ijk[3 * i + 1], ijk[3 * i + 2]};
          nc[a] += sg;
          // a coarser neighbour (any number of levels) is the coarse side's
          // violation, not this leaf's
          bool covered = false;
          for (int k = 0; k <= l && !covered; ++k) {
            int64_t pc[3] = {0, 0, 0};
            for (int b = 0; b < D; ++b) {
              const int64_t n = ncell(l, b);
              pc[b] = (((nc[b] % n) + n) % n) >> k;
            }
            covered = is_leaf(l - k, pc);
          }
          if (covered) continue;
          int tang[2], nt = 0;
          for (int b = 0; b < D; ++b)
            if (b != a) tang[nt++] = b;
          for (int q = 0; q < (1 << (D - 1)); ++q) {
            int64_t ch[3] = {0, 0, 0};
            for (int b = 0; b < D; ++b) {
              const int64_t n = ncell(l, b);
              ch[b] = 2 * (((nc[b] % n) + n) % n);
            }
            ch[a] += sg > 0 ? 0 : 1;
            for (int t = 0; t < nt; ++t) ch[tang[t]] += (q >> t) & 1;
            if (!is_leaf(l + 1, ch)) bad[(size_t)i] = 1;
          }
        }
    }
    return bad;
  }
  void refine(const std::vector<char>& flag) {
    std::vector<int8_t> nl;
    std::vector<int32_t> nc;
    for (size_t c = 0; c < lev.size(); ++c) {
      if (!flag[c]) {
        nl.push_back(lev[c]);
        nc.insert(nc.end(), {ijk[3 * c], ijk[3 * c + 1], ijk[3 * c + 2]});
        continue;
      }
      for (int off = 0; off < (1 << D); ++off) {
        nl.push_back((int8_t)(lev[c] + 1));
        for (int a = 0; a < 3; ++a) nc.push_back(a < D ? 2 * ijk[3 * c + a] + ((off >> a) & 1) : 0);
      }
    }
    lev.swap(nl);
    ijk.swap(nc);
    build_index();
  }
  void morton_sort() {
    int lmax = 0;
    for (int8_t l : lev) lmax = std::max(lmax, (int)l);
    const int64_t C = (int64_t)lev.size();
    std::vector<std::pair<uint64_t, int64_t>> key((size_t)C);
    for (int64_t c = 0; c < C; ++c) {
      uint64_t k = 0;
      const int sh = lmax - lev[c];
      for (int b = 0; b < 21; ++b)
        for (int a = 0; a < D; ++a) k |= (((uint64_t)ijk[3 * c + a] << sh) >> b & 1ull) << (b * D + a);
      key[(size_t)c] = {k, c};
    }
    std::sort(key.begin(), key.end());
    std::vector<int8_t> nl((size_t)C);
    std::vector<int32_t> nc((size_t)C * 3);
    for (int64_t c = 0; c < C; ++c) {
      const int64_t o = key[(size_t)c].second;
      nl[(size_t)c] = lev[(size_t)o];
      for (int a = 0; a < 3; ++a) nc[(size_t)c * 3 + a] = ijk[(size_t)o * 3 + a];
    }
    lev.swap(nl);
    ijk.swap(nc);
    build_index();
  }
};

int octant_of(const int32_t* c, int D) {
  int o = 0;
  for (int a = 0; a < D; ++a) o |= (c[a] & 1) << a;
  return o;
}

}  // namespace

int dg_amr_indicator(dg_handle h, const void* w, uint32_t fields, double* S) {
  if (int r = valid_state(h, w)) return r;
  if (!S) return fail(h, DG_EINVAL, "null S");
  if (h->p.divb != DG_GLM) return fail(h, DG_EUNSUPPORTED, "dynamic refinement is built for the Legendre basis (GLM)");
  if (fields == 0 || fields >= (1u << 9)) return fail(h, DG_EINVAL, "fields: a non-empty mask of the 9 variables");
  h->L->amr_smooth(w, h->g, fields, S, h->stream);
  return check_launch(h, "amr indicator");
}

int dg_amr_plan(dg_handle h, const void* w, uint32_t fields, double s_tilde, int32_t max_level, int64_t* n_new) {
  if (int r = valid_state(h, w)) return r;
  if (!n_new) return fail(h, DG_EINVAL, "null n_new");
  if (h->p.divb != DG_GLM) return fail(h, DG_EUNSUPPORTED, "dynamic refinement is built for the Legendre basis (GLM)");
  if (fields == 0 || fields >= (1u << 9)) return fail(h, DG_EINVAL, "fields: a non-empty mask of the 9 variables");
  if (!(s_tilde > 0.0) || !std::isfinite(s_tilde)) return fail(h, DG_EINVAL, "s_tilde must be positive");
  if (max_level < 0 || max_level > 18) return fail(h, DG_EINVAL, "max_level must be 0..18");
  const int D = h->p.dim, NO = 1 << D;
  const int64_t C = h->g.C;
  LeafSet old;
  old.D = D;
  old.n0[0] = h->g.n0; old.n0[1] = h->g.n1; old.n0[2] = h->g.n2;
  if (!h->h_level.empty()) {
    old.lev = h->h_level;
    old.ijk = h->h_ijk;
  } else {  // uniform grid: level-0 leaves, index i + n0 (j + n1 k)
    old.lev.assign((size_t)C, 0);
    old.ijk.resize((size_t)C * 3);
    for (int64_t c = 0; c < C; ++c) {
      old.ijk[3 * c] = (int32_t)(c % old.n0[0]);
      old.ijk[3 * c + 1] = (int32_t)((c / old.n0[0]) % old.n0[1]);
      old.ijk[3 * c + 2] = (int32_t)(c / (old.n0[0] * old.n0[1]));
    }
  }
  old.build_index();
  // indicators of the leaves
  std::vector<double> S((size_t)C);
  double* dS = nullptr;
  if (int r = check_hip(h, hipMalloc(&dS, (size_t)C * sizeof(double)), "amr S")) return r;
  h->L->amr_smooth(w, h->g, fields, dS, h->stream);
  int rc = check_launch(h, "amr indicator");
  if (!rc) rc = check_hip(h, hipMemcpyAsync(S.data(), dS, (size_t)C * 8, hipMemcpyDeviceToHost, h->stream), "S copy");
  if (!rc) rc = check_hip(h, hipStreamSynchronize(h->stream), "sync");
  (void)hipFree(dS);
  if (rc) return rc;
  std::vector<char> refine((size_t)C, 0);
  for (int64_t c = 0; c < C; ++c) refine[(size_t)c] = (S[(size_t)c] > 2.0 * s_tilde) && old.lev[(size_t)c] < max_level;
  // complete sibling groups with no member marked for refinement
  std::unordered_map<LeafKey, std::vector<int32_t>> groups;
  for (int64_t c = 0; c < C; ++c) {
    const int l = old.lev[(size_t)c];
    if (l == 0) continue;
    const LeafKey pk = leaf_key(l - 1, old.ijk[3 * c] >> 1, old.ijk[3 * c + 1] >> 1, old.ijk[3 * c + 2] >> 1);
    auto& gv = groups[pk];
    if (gv.empty()) gv.assign((size_t)NO, -1);
    gv[(size_t)octant_of(&old.ijk[3 * c], D)] = (int32_t)c;
  }
  std::vector<LeafKey> gkey;
  std::vector<int32_t> gkids;
  for (auto& kv : groups) {
    bool ok = true;
    for (int32_t k : kv.second) ok = ok && k >= 0 && !refine[(size_t)k];
    if (!ok) continue;
    gkey.push_back(kv.first);
    gkids.insert(gkids.end(), kv.second.begin(), kv.second.end());
  }
  const int64_t NG = (int64_t)gkey.size();
  std::vector<double> Sp((size_t)NG);
  if (NG > 0) {
    int32_t* dk = nullptr;
    double* dSp = nullptr;
    rc = check_hip(h, hipMalloc(&dk, gkids.size() * 4), "amr groups");
    if (!rc) rc = check_hip(h, hipMalloc(&dSp, (size_t)NG * 8), "amr Sp");
    if (!rc) rc = check_hip(h, hipMemcpyAsync(dk, gkids.data(), gkids.size() * 4, hipMemcpyHostToDevice, h->stream), "groups");
    if (!rc) {
      h->L->amr_parent_smooth(w, h->g, fields, dk, NG, dSp, h->stream);
      rc = check_launch(h, "amr parent indicator");
    }
    if (!rc) rc = check_hip(h, hipMemcpyAsync(Sp.data(), dSp, (size_t)NG * 8, hipMemcpyDeviceToHost, h->stream), "Sp");
    if (!rc) rc = check_hip(h, hipStreamSynchronize(h->stream), "sync");
    (void)hipFree(dk);
    (void)hipFree(dSp);
    if (rc) return rc;
  }
  std::unordered_map<LeafKey, int64_t> merge;  // parent key -> group row
  for (int64_t gi = 0; gi < NG; ++gi)
    if (Sp[(size_t)gi] < 0.5 * s_tilde) merge.emplace(gkey[(size_t)gi], gi);
  // new leaves; a merge that breaks the 2:1 balance is dropped, the rest is
  // balanced by refinement
  LeafSet nw;
  for (;;) {
    nw = LeafSet();
    nw.D = D;
    for (int a = 0; a < 3; ++a) nw.n0[a] = old.n0[a];
    for (int64_t c = 0; c < C; ++c) {
      const int l = old.lev[(size_t)c];
      const int32_t* x = &old.ijk[3 * c];
      if (l > 0 && merge.count(leaf_key(l - 1, x[0] >> 1, x[1] >> 1, x[2] >> 1))) continue;
      if (refine[(size_t)c]) {
        for (int off = 0; off < NO; ++off) {
          nw.lev.push_back((int8_t)(l + 1));
          for (int a = 0; a < 3; ++a) nw.ijk.push_back(a < D ? 2 * x[a] + ((off >> a) & 1) : 0);
        }
      } else {
        nw.lev.push_back((int8_t)l);
        nw.ijk.insert(nw.ijk.end(), {x[0], x[1], x[2]});
      }
    }
    for (auto& kv : merge) {
      const int32_t* x0 = &old.ijk[3 * (int64_t)gkids[(size_t)kv.second * NO]];
      nw.lev.push_back((int8_t)(old.lev[(size_t)gkids[(size_t)kv.second * NO]] - 1));
      nw.ijk.insert(nw.ijk.end(), {x0[0] >> 1, x0[1] >> 1, x0[2] >> 1});
    }
    nw.build_index();
    const std::vector<char> bad = nw.balance_violations();
    bool dropped = false;
    for (size_t c = 0; c < bad.size(); ++c) {
      if (!bad[c]) continue;
      auto it = merge.find(leaf_key(nw.lev[c], nw.ijk[3 * c], nw.ijk[3 * c + 1], nw.ijk[3 * c + 2]));
      if (it != merge.end()) {
        merge.erase(it);
        dropped = true;
      }
    }
    if (!dropped) break;
  }
  for (int it = 0;; ++it) {
    const std::vector<char> bad = nw.balance_violations();
    bool any = false;
    for (char b : bad) any = any || b;
    if (!any) break;
    if (it >= 20) return fail(h, DG_EINVAL, "amr: 2:1 balance did not converge");
    nw.refine(bad);
  }
  nw.morton_sort();
  // transfer map
  const int64_t NN = (int64_t)nw.lev.size();
  std::vector<int32_t> map((size_t)NN * 4, 0), kids;
  std::unordered_map<int64_t, int32_t> krow;
  for (int64_t i = 0; i < NN; ++i) {
    int l = nw.lev[(size_t)i];
    int64_t x[3] = {nw.ijk[3 * i], nw.ijk[3 * i + 1], nw.ijk[3 * i + 2]};
    auto hit = old.index.find(leaf_key(l, x[0], x[1], x[2]));
    if (hit != old.index.end()) {
      map[4 * i] = 0;
      map[4 * i + 1] = (int32_t)hit->second;
      continue;
    }
    auto mg = merge.find(leaf_key(l, x[0], x[1], x[2]));
    if (mg != merge.end()) {
      auto kr = krow.find(mg->second);
      int32_t row;
      if (kr == krow.end()) {
        row = (int32_t)(kids.size() / NO);
        kids.insert(kids.end(), gkids.begin() + mg->second * NO, gkids.begin() + (mg->second + 1) * NO);
        krow.emplace(mg->second, row);
      } else {
        row = kr->second;
      }
      map[4 * i] = 2;
      map[4 * i + 1] = row;
      continue;
    }
    uint32_t path = 0;
    int depth = 0;
    for (;;) {
      const int32_t cx[3] = {(int32_t)x[0], (int32_t)x[1], (int32_t)x[2]};
      path |= (uint32_t)octant_of(cx, D) << (3 * depth);
      ++depth;
      --l;
      for (int a = 0; a < 3; ++a) x[a] >>= 1;
      if (l < 0 || depth > 10) return fail(h, DG_EINVAL, "amr: a new leaf has no ancestor among the old leaves");
      auto anc = old.index.find(leaf_key(l, x[0], x[1], x[2]));
      if (anc != old.index.end()) {
        map[4 * i] = 1;
        map[4 * i + 1] = (int32_t)anc->second;
        map[4 * i + 2] = depth;
        map[4 * i + 3] = (int32_t)path;  // bits 3k: the octant k levels above the new leaf (top = highest)
        break;
      }
    }
  }
  h->amr_level = nw.lev;
  h->amr_ijk = nw.ijk;
  h->amr_map = map;
  h->amr_kids = kids;
  h->amr_nold = C;
  *n_new = NN;
  return DG_OK;
}

int dg_amr_leaves(dg_handle h, int8_t* level, int32_t* ijk) {
  if (!h) return DG_EINVAL;
  if (h->amr_level.empty()) return fail(h, DG_EINVAL, "no regrid plan: call dg_amr_plan first");
  if (!level || !ijk) return fail(h, DG_EINVAL, "null output");
  std::memcpy(level, h->amr_level.data(), h->amr_level.size());
  std::memcpy(ijk, h->amr_ijk.data(), h->amr_ijk.size() * 4);
  return DG_OK;
}

int dg_amr_transfer(dg_handle h_old, const void* w_old, dg_handle h_new, void* w_new) {
  if (int r = valid_state(h_old, w_old)) return r;
  if (int r = valid_state(h_new, w_new)) return r;
  if (h_old->amr_level.empty()) return fail(h_old, DG_EINVAL, "no regrid plan: call dg_amr_plan first");
  if (h_old->amr_nold != h_old->g.C) return fail(h_old, DG_EINVAL, "the plan belongs to another leaf set");
  if (h_new->p.dim != h_old->p.dim || h_new->p.degree != h_old->p.degree || h_new->p.divb != h_old->p.divb ||
      h_new->p.precision != h_old->p.precision)
    return fail(h_old, DG_EINVAL, "the new handle differs in dimension, degree, scheme or precision");
  if (h_new->h_level != h_old->amr_level || h_new->h_ijk != h_old->amr_ijk)
    return fail(h_old, DG_EINVAL, "the new handle's leaves are not the plan's (dg_amr_leaves)");
  const int NO = 1 << h_old->p.dim;
  const int64_t NN = (int64_t)h_old->amr_level.size();
  int32_t *dmap = nullptr, *dk = nullptr;
  int rc = check_hip(h_old, hipStreamSynchronize(h_old->stream), "sync old");
  if (!rc) rc = check_hip(h_old, hipMalloc(&dmap, h_old->amr_map.size() * 4), "amr map");
  if (!rc) rc = check_hip(h_old, hipMalloc(&dk, std::max<size_t>(h_old->amr_kids.size(), (size_t)NO) * 4), "amr kids");
  if (!rc) rc = check_hip(h_old, hipMemcpy(dmap, h_old->amr_map.data(), h_old->amr_map.size() * 4, hipMemcpyHostToDevice), "map");
  if (!rc && !h_old->amr_kids.empty())
    rc = check_hip(h_old, hipMemcpy(dk, h_old->amr_kids.data(), h_old->amr_kids.size() * 4, hipMemcpyHostToDevice), "kids");
  if (!rc) {
    h_old->L->amr_transfer(w_old, h_old->g.ld, w_new, h_new->g.ld, dmap, dk, NN, h_new->stream);
    rc = check_launch(h_old, "amr transfer");
  }
  if (!rc) rc = check_hip(h_old, hipStreamSynchronize(h_new->stream), "sync new");
  (void)hipFree(dmap);
  (void)hipFree(dk);
  return rc;
}

void dg_destroy(dg_handle h) {
  if (!h) return;
  drop_graph(h);
  h->mlp.release();
  if (h->L) { h->L->free_tables(); delete h->L; }
  if (h->ff) (void)hipFree(h->ff);
  if (h->jp) (void)hipFree(h->jp);
  if (h->jsum) (void)hipFree(h->jsum);
  if (h->S1) (void)hipFree(h->S1);
  if (h->S2) (void)hipFree(h->S2);
  if (h->S3) (void)hipFree(h->S3);
  if (h->lscr) (void)hipFree(h->lscr);
  if (h->sc) (void)hipFree(h->sc);
  for (void* q : h->mesh_bufs) (void)hipFree(q);
  delete h;
}

}  // extern "C"
