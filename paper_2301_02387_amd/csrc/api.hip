// C ABI of the hot path: handles, device memory, and the orchestration of
// the kernels for each entry point declared in include/mh.h.  An operator
// handle holds a batch of instances (a plain operator is a batch of one);
// every kernel launch covers all of them (kernels.hpp).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <memory>
#include <mutex>
#include <new>
#include <string>
#include <thread>
#include <vector>

#include "../../include/mh.h"
#include "host.hpp"
#include "adjoint.hpp"
#include "kernels.hpp"
#include "mg.hpp"

using namespace mh;

namespace {

thread_local std::string g_err;
thread_local std::string g_alloc_detail;  // what the last failed allocation asked for

int fail(int code, const std::string& msg) {
  g_err = msg;
  return code;
}

// Device buffers: from the registered allocator (mh_set_allocator) or
// hipMalloc; each remembers the pair that made it.
struct AllocHook {
  mh_alloc_fn alloc = nullptr;
  mh_free_fn free = nullptr;
  void* ctx = nullptr;
};
AllocHook g_hook;
struct DevBlock {
  void* p = nullptr;
  size_t bytes = 0;
  AllocHook hook;
};
DevBlock dev_alloc(size_t bytes) {
  DevBlock b;
  b.bytes = bytes;
  b.hook = g_hook;
  if (b.hook.alloc) {
    b.p = b.hook.alloc(bytes, b.hook.ctx);
    if (!b.p) {
      g_alloc_detail = "registered allocator (" + std::to_string(bytes) + " bytes)";
      throw std::bad_alloc();
    }
  } else {
    hipError_t e = hipMalloc(&b.p, bytes);
    if (e != hipSuccess) {
      g_alloc_detail = "hipMalloc(" + std::to_string(bytes) + " bytes): " + hipGetErrorString(e);
      throw std::bad_alloc();
    }
  }
  return b;
}
void dev_free(const DevBlock& b) {
  if (!b.p) return;
  if (b.hook.free) b.hook.free(b.p, b.bytes, b.hook.ctx);
  else (void)hipFree(b.p);
}

struct HipError {
  hipError_t e;
  const char* what;
};

#define HIPCHK(x)                                  \
  do {                                             \
    hipError_t _e = (x);                           \
    if (_e != hipSuccess) throw HipError{_e, #x};  \
  } while (0)

}  // namespace

struct mh_mesh {
  Mesh M;
};

struct mh_op {
  int ni = 1;                  // instances
  int device = 0;              // HIP device current at creation (all its buffers live there)
  std::vector<Mesh> Ms;        // per instance
  std::vector<OpHost> Hs;
  std::vector<DevMesh> dh;     // host copies of the device instance records
  DevMesh* dm = nullptr;       // device [ni]
  Batch B;
  std::vector<DevBlock> allocs;
  int n = 0, ncol = 0, lmax = 12;
  double rtol = 1e-12, rdm_eps = 1e-10;
  double krylov_tol = 0.0;     // error threshold of the adaptive Krylov dimension (0: fixed dimension)
  int maxit = 5000;
  // device data
  int* colinfo = nullptr;  // per real Poisson column: r | s<<8 | part<<16
  int* colmap = nullptr;   // [n*n]: first column of pair (r<=s)
  double* Ebuf = nullptr;  // [2]: field value of the frozen operator, field value of a load-vector call
  // orbital workspaces (batch arrays over extended rows, or [ni][...] small blocks)
  double* acc = nullptr;    // [tE][n] c128
  double* Upk = nullptr;    // [tE][n*n]
  double* ginv = nullptr;   // [ni][n][n] c128
  double* lam = nullptr;    // [ni][n][n] c128
  double* F = nullptr;      // [tE][n] c128
  double* kq = nullptr;     // [tE][n] c128: assembled stiffness times the orbitals (orbital schedule bit 2)
  double* kred = nullptr;   // [ni][RED_SLOTS][2n] scratch accumulators of that operator pass
  double* ma_b = nullptr, *ma_x = nullptr, *ma_r = nullptr, *ma_d0 = nullptr, *ma_d1 = nullptr;  // [tMa][n]
  double* gpart = nullptr;  // reduction partials
  double* Mr = nullptr;     // [ni][n^2][n^2]
  double* Gtmp = nullptr;   // [ni][n^2][n^2] c128
  int* flag = nullptr;      // [ni]
  // multigrid preconditioner of the Poisson solves (built on first use)
  std::unique_ptr<MgDev> mg;
  double* mg_red = nullptr;   // scratch accumulators of the level-0 operator passes
  int* cg_done = nullptr;     // [ni] convergence flags of a batch's multigrid CG (zero outside it)
  double* mg_part = nullptr;  // r.z partials
  int mg_levels = 0;
  int cg_hint = 0;            // iterations of the last multigrid-preconditioned solve
  bool frozen = false;
  // Krylov
  int m_alloc = 0;
  std::vector<double*> V;   // host list of device vectors
  double** Vdev = nullptr;  // device pointer table
  Krylov K;
  // Poisson
  PoissonWs P;
  // CI
  CIDev ci;
  int na = 0, nb = 0;
  std::vector<double*> Qh;
  double** Qdev = nullptr;
  Krylov KC;
  double* gam = nullptr, *Gam = nullptr, *hmat = nullptr, *gint = nullptr, *S = nullptr, *zmat = nullptr;
  double* pmat = nullptr;   // [ni][n][n] c128: <phi_p| -i S_e |phi_q> (momentum along e)
  double* obs = nullptr;    // [ni][8]
  double* Rinv = nullptr;
  double* Wprev = nullptr;  // [tF][n*n] potentials of the previous step (start extrapolation)
  double* Wprev2 = nullptr; // [tF][n*n] and of the step before
  double* hostpin = nullptr;
  size_t hostpin_len = 0;
  hipStream_t gstream = nullptr;  // stream for graph capture and replay
  double* Etab = nullptr;         // field values of a propagation call (whole-step graph replay)
  int64_t Etab_len = 0;
  int* step_ctr = nullptr;        // device step counter of the replayed steps
  // timing of the dominant kernels: pools of event pairs recorded on the
  // launch stream around each launch (no synchronisation while recording)
  std::vector<hipEvent_t> ev[2];
  int ev_used[2] = {0, 0};
  bool timing = false;

  template <class T>
  T* alloc(size_t count) {
    const DevBlock b = dev_alloc(std::max<size_t>(count * sizeof(T), 16));
    allocs.push_back(b);
    return (T*)b.p;
  }
  void release(void* p) {  // one buffer back to the allocator that made it
    for (size_t i = 0; i < allocs.size(); ++i)
      if (allocs[i].p == p) {
        dev_free(allocs[i]);
        allocs.erase(allocs.begin() + i);
        return;
      }
  }
  template <class T>
  T* upload(const std::vector<T>& v, hipStream_t s) {
    T* p = alloc<T>(v.size());
    if (!v.empty()) HIPCHK(hipMemcpyAsync(p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, s));
    return p;
  }
  ~mh_op() {
    (void)hipDeviceSynchronize();  // no kernel still uses a buffer handed back
    for (const DevBlock& b : allocs) dev_free(b);
    for (int k = 0; k < 2; ++k)
      for (hipEvent_t e : ev[k]) (void)hipEventDestroy(e);
    if (hostpin) (void)hipHostFree(hostpin);
    if (gstream) (void)hipStreamDestroy(gstream);
  }
};

static inline hipStream_t S(void* s) { return (hipStream_t)s; }
// largest interface block held as a dense inverse (doubles: MA_DENSE_MAX^2 x 8 B = 128 MiB)
constexpr int64_t MA_DENSE_MAX = 4096;

template <class F>
static int guarded(F&& f) {
  try {
    return f();
  } catch (const HipError& e) {
    return fail(MH_HIP_ERROR, std::string("HIP error ") + hipGetErrorString(e.e) + " in " + e.what);
  } catch (const std::bad_alloc&) {
    std::string d = g_alloc_detail;
    g_alloc_detail.clear();
    return fail(MH_OOM, "device or host allocation failed" + (d.empty() ? std::string() : ": " + d));
  } catch (const std::exception& e) {
    return fail(MH_INVALID_ARG, e.what());
  } catch (...) {
    return fail(MH_INVALID_ARG, "unknown error");
  }
}

extern "C" const char* mh_last_error(void) { return g_err.c_str(); }

extern "C" int mh_set_allocator(mh_alloc_fn alloc_fn, mh_free_fn free_fn, void* ctx) {
  if ((alloc_fn == nullptr) != (free_fn == nullptr)) return fail(MH_INVALID_ARG, "give both allocator functions or neither");
  g_hook.alloc = alloc_fn;
  g_hook.free = free_fn;
  g_hook.ctx = alloc_fn ? ctx : nullptr;
  return MH_OK;
}

// ------------------------------------------------------------------ mesh ----
extern "C" int mh_mesh_create(const mh_mesh_desc* desc, mh_mesh** out) {
  if (!desc || !out) return fail(MH_INVALID_ARG, "null argument");
  if (desc->n_balls < 0 || (desc->n_balls > 0 && !desc->balls)) return fail(MH_INVALID_ARG, "bad balls");
  if (desc->n_kelly < 0 || (desc->n_kelly > 0 && !desc->kelly_nuclei)) return fail(MH_INVALID_ARG, "bad Kelly nuclei");
  return guarded([&]() -> int {
    std::vector<Ball> balls;
    for (int i = 0; i < desc->n_balls; ++i) {
      Ball b;
      for (int d = 0; d < 3; ++d) b.c[d] = desc->balls[i].center[d];
      b.r = desc->balls[i].radius;
      b.levels = desc->balls[i].levels;
      balls.push_back(b);
    }
    KellyReq kr;
    for (int i = 0; i < desc->n_kelly; ++i) {
      Nucleus n;
      n.Z = desc->kelly_nuclei[4 * i];
      for (int d = 0; d < 3; ++d) n.R[d] = desc->kelly_nuclei[4 * i + 1 + d];
      kr.nuclei.push_back(n);
    }
    kr.tol = desc->kelly_tol;
    kr.soft = desc->kelly_soft;
    kr.max_level = desc->kelly_max_level;
    auto m = std::make_unique<mh_mesh>();
    bool unsup = false;
    std::string err = build_mesh(desc->lo, desc->hi, desc->n_coarse, desc->p, balls, m->M, unsup, &kr);
    if (!err.empty()) return fail(unsup ? MH_UNSUPPORTED : MH_INVALID_ARG, err);
    *out = m.release();
    return MH_OK;
  });
}

extern "C" int mh_mesh_info_get(const mh_mesh* mesh, mh_mesh_info* info) {
  if (!mesh || !info) return fail(MH_INVALID_ARG, "null argument");
  const Mesh& M = mesh->M;
  std::memset(info, 0, sizeof(*info));
  info->n_cells = M.n_cells;
  info->n_full = M.nF;
  info->n_dof = M.N;
  info->n_hang = M.Nh;
  info->n_bnd = M.Nb;
  info->n_masters = (int64_t)M.masters.size();
  info->hang_nnz = (int64_t)M.hang_col.size();
  info->p = M.p;
  info->max_level = M.Lmax;
  for (int l = 0; l <= M.Lmax && l < 16; ++l) info->level_counts[l] = M.level_counts[l];
  info->kelly_rounds = M.kelly_rounds;
  return MH_OK;
}

extern "C" int mh_mesh_node_coords(const mh_mesh* mesh, double* xyz) {
  if (!mesh || !xyz) return fail(MH_INVALID_ARG, "null argument");
  std::memcpy(xyz, mesh->M.xyz.data(), mesh->M.xyz.size() * sizeof(double));
  return MH_OK;
}

extern "C" int mh_mesh_constraints(const mh_mesh* mesh, int64_t* ptr, int64_t* col, double* w) {
  if (!mesh) return fail(MH_INVALID_ARG, "null argument");
  const Mesh& M = mesh->M;
  if (ptr) std::memcpy(ptr, M.hang_ptr.data(), M.hang_ptr.size() * sizeof(int64_t));
  if (col) std::memcpy(col, M.hang_col.data(), M.hang_col.size() * sizeof(int64_t));
  if (w) std::memcpy(w, M.hang_w.data(), M.hang_w.size() * sizeof(double));
  return MH_OK;
}

extern "C" int mh_mesh_cells(const mh_mesh* mesh, int32_t* nodes, int32_t* level, double* origin) {
  if (!mesh) return fail(MH_INVALID_ARG, "null argument");
  const Mesh& M = mesh->M;
  if (nodes) std::memcpy(nodes, M.cell_nodes.data(), M.cell_nodes.size() * sizeof(int32_t));
  if (level) std::memcpy(level, M.cell_level.data(), M.cell_level.size() * sizeof(int32_t));
  if (origin) std::memcpy(origin, M.cell_org.data(), M.cell_org.size() * sizeof(double));
  return MH_OK;
}

extern "C" int mh_mesh_destroy(mh_mesh* mesh) {
  delete mesh;
  return MH_OK;
}

// -------------------------------------------------------------- operator ----
static int popcount32(uint32_t x) { return __builtin_popcount(x); }

// a+_p a_q on string s: returns sign (0 if impossible) and the new string
static int excite(uint32_t s, int p, int q, uint32_t* out) {
  if (!((s >> q) & 1u)) return 0;
  int sign = (popcount32(s & ((1u << q) - 1u)) & 1) ? -1 : 1;
  uint32_t s2 = s & ~(1u << q);
  if ((s2 >> p) & 1u) return 0;
  if (popcount32(s2 & ((1u << p) - 1u)) & 1) sign = -sign;
  *out = s2 | (1u << p);
  return sign;
}

static std::vector<uint32_t> make_strings(int n, int k) {
  std::vector<uint32_t> v;
  for (uint32_t s = 0; s < (1u << n); ++s)
    if (popcount32(s) == k) v.push_back(s);
  return v;
}

// table[J][p*n+q] = I | (sign<0)<<30 with E_pq |I> = sign |J> (from E_qp |J>)
static std::vector<int32_t> excitation_table(int n, const std::vector<uint32_t>& str) {
  std::vector<int32_t> idx(1u << n, -1);
  for (size_t i = 0; i < str.size(); ++i) idx[str[i]] = (int32_t)i;
  std::vector<int32_t> t(str.size() * n * n, -1);
  for (size_t J = 0; J < str.size(); ++J)
    for (int p = 0; p < n; ++p)
      for (int q = 0; q < n; ++q) {
        uint32_t I = 0;
        int sg = excite(str[J], q, p, &I);
        if (sg) t[J * n * n + p * n + q] = idx[I] | (sg < 0 ? (1 << 30) : 0);
      }
  return t;
}

static void krylov_alloc(mh_op* op, Krylov& K, int m_max, int nblk) {
  const size_t ni = op->ni;
  K.m_max = m_max;
  K.H = op->alloc<double>(ni * 2 * (m_max + 1) * m_max);
  K.hcur = op->alloc<double>(ni * 2 * (m_max + 1));
  K.scal = op->alloc<double>(ni * 8);
  K.y = op->alloc<double>(ni * 2 * m_max);
  K.nblk = nblk;
  K.part = op->alloc<double>(ni * (size_t)nblk * (2 * (m_max + 1) + 1) + 64);
}

// Per-instance Chebyshev coefficients for `iters` iterations from that
// instance's spectrum bounds: 1/theta, then (rho_{k+1} rho_k, 2 rho_{k+1}/delta).
static std::vector<double> cheb_table(double lo, double hi, int iters, bool used) {
  std::vector<double> t(1 + 2 * (size_t)iters, 0.0);
  if (!used) return t;
  const double theta = 0.5 * (hi + lo), delta = 0.5 * (hi - lo), sigma = theta / delta;
  t[0] = 1.0 / theta;
  double rho = 1.0 / sigma;
  for (int k = 0; k < iters; ++k) {
    const double rho1 = 1.0 / (2.0 * sigma - rho);
    t[1 + 2 * k] = rho1 * rho;
    t[2 + 2 * k] = 2.0 * rho1 / delta;
    rho = rho1;
  }
  return t;
}

struct InstanceSpec {
  const Mesh* mesh;
  std::vector<Nucleus> nuc;
  double pol[3];
  double E0;
  EcsReq ecs;
};

static double nuclear_repulsion(const std::vector<Nucleus>& nuc) {
  double vnn = 0.0;
  for (size_t a = 0; a < nuc.size(); ++a)
    for (size_t b = a + 1; b < nuc.size(); ++b) {
      double dx = nuc[a].R[0] - nuc[b].R[0], dy = nuc[a].R[1] - nuc[b].R[1], dz = nuc[a].R[2] - nuc[b].R[2];
      vnn += nuc[a].Z * nuc[b].Z / std::sqrt(dx * dx + dy * dy + dz * dz);
    }
  return vnn;
}

static void upload_instances(mh_op* op, hipStream_t s) {
  HIPCHK(hipMemcpyAsync(op->dm, op->dh.data(), op->dh.size() * sizeof(DevMesh), hipMemcpyHostToDevice, s));
  HIPCHK(hipStreamSynchronize(s));
  op->B.mx.sched_orb = op->dh[0].sched_orb;
  op->B.mx.sched_poi = op->dh[0].sched_poi;
  op->B.mx.grid_orb = op->dh[0].grid_orb;
  op->B.mx.grid_poi = op->dh[0].grid_poi;
}

// Build the host operators of all instances (in parallel), upload them and
// allocate the batch workspaces.
// Device scratch of the allocation-free mass solve (mh_mass_solve_noalloc):
// the interface system's gathered right-hand side, iterate, residual and two
// Chebyshev directions, laid out one after another.  Every GPU the library
// runs on holds one copy until the process ends.  In host code `scratch`
// names a host-side stand-in, never the device memory: its device address is
// taken once per device with hipGetSymbolAddress (with that device current,
// when an operator is created there) and kept in g_scratch_dev.
constexpr size_t kScratchBytes = size_t(32) << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {
std::mutex g_scratch_mu;
std::vector<void*> g_scratch_dev;  // device address of `scratch` per device id (nullptr: not yet taken)

// Device address of the scratch array on the current device, taken on first use.
int resolve_scratch() {
  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if ((int)g_scratch_dev.size() <= dev) g_scratch_dev.resize(dev + 1, nullptr);
  if (!g_scratch_dev[dev]) {
    void* ptr = nullptr;
    HIPCHK(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
    g_scratch_dev[dev] = ptr;
  }
  return dev;
}

void* scratch_on(int dev) {
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  return dev < (int)g_scratch_dev.size() ? g_scratch_dev[dev] : nullptr;
}
}  // namespace

static mh_op* create_batch(const std::vector<InstanceSpec>& spec, const mh_op_desc& desc, hipStream_t s) {
  const int ni = (int)spec.size();
  const int n = desc.n_orb, ncol = n * n;
  const int lmax = desc.lmax_bc > 0 ? desc.lmax_bc : 12;
  // Bring up the HIP runtime (device discovery and its address reservations)
  // before the set-up threads start.
  HIPCHK(hipFree(nullptr));
  auto op = std::make_unique<mh_op>();
  op->ni = ni;
  op->device = resolve_scratch();
  op->Ms.resize(ni);
  op->Hs.resize(ni);
  {
    const int nthr = std::max(1, std::min<int>(ni, std::min(16u, std::max(1u, std::thread::hardware_concurrency()))));
    std::vector<std::thread> pool;
    std::vector<std::string> errs(nthr);
    for (int t = 0; t < nthr; ++t)
      pool.emplace_back([&, t]() {
        try {
          for (int i = t; i < ni; i += nthr) {
            op->Ms[i] = *spec[i].mesh;
            build_operator(op->Ms[i], spec[i].nuc, spec[i].pol, lmax, op->Hs[i], &spec[i].ecs);
          }
        } catch (const std::exception& e) {
          errs[t] = e.what();
        }
      });
    for (auto& th : pool) th.join();
    for (auto& e : errs)
      if (!e.empty()) throw std::runtime_error(e);
  }
  op->n = n;
  op->ncol = ncol;
  op->lmax = lmax;
  op->rtol = desc.poisson_rtol > 0 ? desc.poisson_rtol : 1e-12;
  op->maxit = desc.poisson_maxit > 0 ? desc.poisson_maxit : 5000;
  op->rdm_eps = desc.rdm_eps > 0 ? desc.rdm_eps : 1e-10;
  op->krylov_tol = desc.krylov_tol;
  Batch& B = op->B;
  B.ni = ni;
  int iters = 0;
  for (int i = 0; i < ni; ++i)
    if (!op->Ms[i].masters.empty()) iters = std::max(iters, op->Hs[i].cheb_iters);
  B.cheb_iters = iters;
  op->dh.resize(ni);
  DevMesh& mx = B.mx;
  int64_t oE = 0, oF = 0, oMa = 0;
  std::vector<std::vector<float>> keep_f;
  keep_f.reserve(ni);
  for (int i = 0; i < ni; ++i) {
    const Mesh& M = op->Ms[i];
    const OpHost& H = op->Hs[i];
    DevMesh& d = op->dh[i];
    d.P = M.P;
    d.n = n;
    d.inst = i;
    d.nC = M.n_cells;
    d.N = M.N;
    d.NE = M.N + M.Nh;
    d.NF = M.nF;
    d.Nh = M.Nh;
    d.Nb = M.Nb;
    d.nMa = (int64_t)M.masters.size();
    d.oE = oE;
    d.oF = oF;
    d.oMa = oMa;
    oE += d.NE;
    oF += d.NF;
    oMa += d.nMa;
    d.cell_nodes = op->upload(M.cell_nodes, s);
    std::vector<double> hh(M.n_cells);
    for (int64_t e = 0; e < M.n_cells; ++e) hh[e] = 0.5 * M.cell_h[e];
    d.cell_hh = op->upload(hh, s);
    d.m = op->upload(H.m, s);
    d.v = op->upload(H.v, s);
    d.mz = op->upload(H.mz, s);
    d.xyz = op->upload(M.xyz, s);
    std::vector<int32_t> hp(M.hang_ptr.begin(), M.hang_ptr.end()), hc(M.hang_col.begin(), M.hang_col.end());
    d.hang_ptr = op->upload(hp, s);
    d.hang_col = op->upload(hc, s);
    d.hang_w = op->upload(M.hang_w, s);
    d.ma_index = op->upload(H.ma_index, s);
    d.ma_dof = op->upload(H.ma_dof, s);
    d.ma_ptr = op->upload(H.ma_ptr, s);
    d.ma_col = op->upload(H.ma_col, s);
    d.ma_val = op->upload(H.ma_val, s);
    d.ma_dinv = op->upload(H.ma_dinv, s);
    d.cheb = op->upload(cheb_table(H.cheb_lo, H.cheb_hi, iters, d.nMa > 0), s);
    d.ct_ptr = op->upload(H.ct_ptr, s);
    d.ct_row = op->upload(H.ct_row, s);
    d.ct_w = op->upload(H.ct_w, s);
    d.inv_mass = op->upload(H.inv_mass, s);
    d.kdiag_inv = op->upload(H.kdiag_inv, s);
    d.node_inc = op->upload(H.node_inc, s);
    d.kt_ptr = op->upload(H.kt_ptr, s);
    d.kt_col = op->upload(H.kt_col, s);
    d.kt_val = op->upload(H.kt_val, s);
    keep_f.emplace_back(H.kt_val.begin(), H.kt_val.end());   // host copy alive until the final synchronisation
    d.kt_valf = op->upload(keep_f.back(), s);
    {
      std::vector<int32_t> lr;
      for (int64_t r = 0; r < d.N; ++r)
        if (H.kt_ptr[r + 1] - H.kt_ptr[r] > KT_LONG) lr.push_back((int32_t)r);
      d.kt_long = op->upload(lr, s);
      d.n_long = (int64_t)lr.size();
    }
    d.bnd_cells = op->upload(H.bnd_cells, s);
    d.n_bnd_cells = (int64_t)H.bnd_cells.size();
    d.bnd_table = op->upload(H.bnd_table, s);
    for (int k = 0; k < 3; ++k) d.center[k] = 0.5 * (M.lo + M.hi);
    d.E0 = spec[i].E0;
    d.vnn = nuclear_repulsion(spec[i].nuc);
    for (int k = 0; k < 16; ++k) d.A[k] = 0.0;
    for (int k = 0; k < 4; ++k) d.w[k] = 0.0;
    for (int k = 0; k < 16; ++k) d.Qs[k] = 0.0;
    for (int a = 0; a < M.P; ++a) {
      d.w[a] = M.gll.w[a];
      for (int b = 0; b < M.P; ++b) {
        d.A[a * M.P + b] = M.gll.A[a * M.P + b];
        d.Qs[a * M.P + b] = M.gll.Qs[a * M.P + b];
      }
    }
    for (int k = 0; k < 3; ++k) d.pol[k] = spec[i].pol[k];
    d.gauge = desc.gauge;
    if (H.ecs) {
      d.ecs = 1;
      d.ecs_code = op->upload(H.ecs_code, s);
      d.ecs_rho = op->upload(H.ecs_rho, s);
      d.ecs_v = op->upload(H.ecs_v, s);
      d.ecs_mz = op->upload(H.ecs_mz, s);
      for (int k = 0; k < 6; ++k) {
        d.ecs_pw[2 * k] = std::cos((k - 2) * H.ecs_theta);
        d.ecs_pw[2 * k + 1] = std::sin((k - 2) * H.ecs_theta);
      }
    }
    if (i == 0) mx = d;
    mx.ecs = std::max(mx.ecs, d.ecs);
    mx.nC = std::max(mx.nC, d.nC);
    mx.N = std::max(mx.N, d.N);
    mx.NE = std::max(mx.NE, d.NE);
    mx.NF = std::max(mx.NF, d.NF);
    mx.Nh = std::max(mx.Nh, d.Nh);
    mx.Nb = std::max(mx.Nb, d.Nb);
    mx.nMa = std::max(mx.nMa, d.nMa);
    mx.n_bnd_cells = std::max(mx.n_bnd_cells, d.n_bnd_cells);
    mx.n_long = std::max(mx.n_long, d.n_long);
    if (d.P != mx.P) throw std::runtime_error("all instances of a batch must use the same degree p");
  }
  B.tE = oE;
  B.tF = oF;
  B.tMa = oMa;
  // one instance with a small interface block: its dense inverse (SPD,
  // Gauss-Jordan on the device), so each interface solve is one matrix-vector
  // pass instead of a chain of Chebyshev launches
  if (ni == 1 && op->dh[0].nMa > 0 && op->dh[0].nMa <= MA_DENSE_MAX) {
    const OpHost& H = op->Hs[0];
    const int64_t nm = op->dh[0].nMa;
    std::vector<double> A((size_t)(nm * nm), 0.0);
    for (int64_t i = 0; i < nm; ++i)
      for (int32_t t = H.ma_ptr[i]; t < H.ma_ptr[i + 1]; ++t) A[(size_t)(i * nm + H.ma_col[t])] += H.ma_val[t];
    double* Ad = op->upload(A, s);
    HIPCHK(hipStreamSynchronize(s));  // A is a host temporary
    launch_dense_inverse(Ad, nm, s);
    op->dh[0].ma_inv = Ad;
    mx.ma_inv = Ad;
  }
  op->dm = op->alloc<DevMesh>(ni);
  B.dm = op->dm;
  upload_instances(op.get(), s);
  // Poisson column layout
  std::vector<int> colinfo, colmap(n * n, -1);
  for (int r = 0; r < n; ++r)
    for (int q = r; q < n; ++q) {
      colmap[r * n + q] = (int)colinfo.size();
      colinfo.push_back(r | (q << 8));
      if (q != r) colinfo.push_back(r | (q << 8) | (1 << 16));
    }
  op->colinfo = op->upload(colinfo, s);
  op->colmap = op->upload(colmap, s);
  op->Ebuf = op->alloc<double>(2);
  launch_zero(op->Ebuf, 2, s);
  // orbital workspaces
  const size_t tE = B.tE, nn = (size_t)n * n, n4 = nn * nn;
  op->acc = op->alloc<double>(2 * tE * n);
  launch_zero(op->acc, 2 * tE * n, s);
  op->Upk = op->alloc<double>(tE * nn);
  op->ginv = op->alloc<double>(ni * 2 * nn);
  op->lam = op->alloc<double>(ni * 2 * nn);
  op->F = op->alloc<double>(2 * tE * n);
  op->kq = op->alloc<double>(2 * tE * n);
  op->kred = op->alloc<double>((size_t)ni * RED_SLOTS * 2 * n);
  const size_t nma = std::max<size_t>(1, B.tMa);
  op->ma_b = op->alloc<double>(2 * nma * n);
  op->ma_x = op->alloc<double>(2 * nma * n);
  op->ma_r = op->alloc<double>(2 * nma * n);
  op->ma_d0 = op->alloc<double>(2 * nma * n);
  op->ma_d1 = op->alloc<double>(2 * nma * n);
  const int gblk = std::max(gram_blocks(mx.NE), gint_blocks(B));
  op->gpart = op->alloc<double>((size_t)ni * gblk * 2 * std::max(nn, n4) + 64);
  op->Mr = op->alloc<double>(ni * n4);
  op->Gtmp = op->alloc<double>(ni * 2 * n4);
  op->flag = op->alloc<int>(ni);
  op->gam = op->alloc<double>(ni * 2 * nn);
  op->Gam = op->alloc<double>(ni * 2 * n4);
  op->hmat = op->alloc<double>(ni * 2 * nn);
  op->gint = op->alloc<double>(ni * 2 * n4);
  op->S = op->alloc<double>(ni * 2 * nn);
  op->zmat = op->alloc<double>(ni * 2 * nn);
  op->pmat = op->alloc<double>(ni * 2 * nn);
  op->obs = op->alloc<double>(ni * 8);
  op->Rinv = op->alloc<double>(ni * 2 * nn);
  op->hostpin_len = (size_t)ni * std::max((8 + RED_SLOTS) * ncol, 64) + 4096;
  HIPCHK(hipHostMalloc((void**)&op->hostpin, op->hostpin_len * sizeof(double), hipHostMallocDefault));
  // Poisson workspaces
  PoissonWs& P = op->P;
  P.ncol = ncol;
  P.lmax = lmax;
  P.nharm = (lmax + 1) * (lmax + 1);
  P.acc = op->alloc<double>(tE * ncol);
  launch_zero(P.acc, tE * ncol, s);
  P.p = op->alloc<double>(tE * ncol);
  launch_zero(P.p, tE * ncol, s);
  P.p2 = op->alloc<double>(tE * ncol);
  launch_zero(P.p2, tE * ncol, s);
  P.r = op->alloc<double>(tE * ncol);
  P.q = op->alloc<double>(tE * ncol);
  P.sc = op->alloc<double>((size_t)ni * 8 * ncol);
  launch_zero(P.sc, (size_t)ni * 8 * ncol, s);
  P.red = op->alloc<double>((size_t)ni * RED_SLOTS * ncol);
  launch_zero(P.red, (size_t)ni * RED_SLOTS * ncol, s);
  if (ni == 1) {  // the largest operator-pass grid (65,536 sweeping and up to 2,056 long-row workgroups)
    B.spart_cap = (int64_t)(65536 + 4096) * std::max(ncol, 2 * n);
    B.spart = op->alloc<double>((size_t)B.spart_cap);
  }
  P.part_stride = (int64_t)8192 * 2 * ncol;
  P.part = op->alloc<double>((size_t)ni * P.part_stride);
  P.Q = op->alloc<double>((size_t)ni * P.nharm * ncol);
  // moment partial sums: up to 2048 workgroups on the matrix-core form (16 or more columns), 512 otherwise
  P.mblk = (int)std::min<int64_t>(ncol >= 16 ? 2048 : 512, std::max<int64_t>(1, (mx.NE + 31) / 32));
  P.mpart = op->alloc<double>((size_t)ni * P.mblk * P.nharm * ncol);
  // CI space
  op->na = desc.n_alpha;
  op->nb = desc.n_beta;
  auto sa = make_strings(n, desc.n_alpha), sb = make_strings(n, desc.n_beta);
  CIDev& c = op->ci;
  c.n = n;
  c.NA = (int)sa.size();
  c.NB = (int)sb.size();
  c.dim = c.NA * c.NB;
  c.exa = op->upload(excitation_table(n, sa), s);
  c.exb = op->upload(excitation_table(n, sb), s);
  c.D = op->alloc<double>((size_t)ni * 2 * c.dim * ncol);
  c.T = op->alloc<double>((size_t)ni * 2 * c.dim * ncol);
  c.hp = op->alloc<double>((size_t)ni * 2 * ncol);
  c.w = op->alloc<double>((size_t)ni * 2 * c.dim);
  c.part = op->alloc<double>((size_t)ni * gram_blocks(c.dim) * 2 * 4096 + 64);
  int mci = std::min(12, c.dim);
  for (int j = 0; j <= mci; ++j) op->Qh.push_back(op->alloc<double>((size_t)ni * 2 * c.dim));
  op->Qdev = op->alloc<double*>(op->Qh.size());
  HIPCHK(hipMemcpyAsync(op->Qdev, op->Qh.data(), op->Qh.size() * sizeof(double*), hipMemcpyHostToDevice, s));
  krylov_alloc(op.get(), op->KC, 12, 1);
  HIPCHK(hipStreamSynchronize(s));
  return op.release();
}

static int check_desc(const mh_op_desc* desc) {
  if (desc->n_orb < 1 || desc->n_orb > 8) return fail(MH_UNSUPPORTED, "n_orb must be 1..8");
  if (desc->n_alpha < 0 || desc->n_beta < 0 || desc->n_alpha > desc->n_orb || desc->n_beta > desc->n_orb ||
      desc->n_alpha + desc->n_beta < 1)
    return fail(MH_INVALID_ARG, "electron counts");
  if (desc->n_nuclei < 0 || (desc->n_nuclei > 0 && (!desc->charges || !desc->positions)))
    return fail(MH_INVALID_ARG, "nuclei");
  const int lmax = desc->lmax_bc > 0 ? desc->lmax_bc : 12;
  if (lmax > 12) return fail(MH_UNSUPPORTED, "lmax_bc must be <= 12");
  if (desc->gauge != MH_GAUGE_LENGTH && desc->gauge != MH_GAUGE_VELOCITY) return fail(MH_INVALID_ARG, "gauge");
  if (!(desc->krylov_tol >= 0.0)) return fail(MH_INVALID_ARG, "krylov_tol must be >= 0");
  if (!(desc->ecs_theta >= 0.0 && desc->ecs_theta < 1.5707963267948966))
    return fail(MH_INVALID_ARG, "ecs_theta must lie in [0, pi/2)");
  if (desc->ecs_theta > 0.0)
    for (int d = 0; d < 3; ++d)
      if (!(desc->ecs_inner[d] >= 0.0)) return fail(MH_INVALID_ARG, "ecs_inner must be >= 0");
  if ((lmax + 1) * (lmax + 1) * desc->n_orb * desc->n_orb > 48 * 256)
    return fail(MH_UNSUPPORTED, "multipole table too large");
  return MH_OK;
}

static InstanceSpec make_spec(const mh_mesh* mesh, const mh_op_desc* desc, double E0) {
  InstanceSpec sp;
  sp.mesh = &mesh->M;
  for (int i = 0; i < desc->n_nuclei; ++i) {
    Nucleus a;
    a.Z = desc->charges[i];
    for (int k = 0; k < 3; ++k) a.R[k] = desc->positions[3 * i + k];
    sp.nuc.push_back(a);
  }
  for (int k = 0; k < 3; ++k) sp.pol[k] = desc->polarization[k];
  sp.E0 = E0;
  sp.ecs.theta = desc->ecs_theta;
  for (int k = 0; k < 3; ++k) sp.ecs.inner[k] = desc->ecs_inner[k];
  return sp;
}

extern "C" int mh_op_create(const mh_mesh* mesh, const mh_op_desc* desc, void* stream, mh_op** out) {
  if (!mesh || !desc || !out) return fail(MH_INVALID_ARG, "null argument");
  int rc = check_desc(desc);
  if (rc != MH_OK) return rc;
  return guarded([&]() -> int {
    std::vector<InstanceSpec> spec{make_spec(mesh, desc, 1.0)};
    *out = create_batch(spec, *desc, S(stream));
    return MH_OK;
  });
}

extern "C" int mh_batch_create(const mh_mesh* const* meshes, const mh_op_desc* descs, const double* field_scale,
                               int32_t n_inst, void* stream, mh_op** out) {
  if (!meshes || !descs || !out || n_inst < 1) return fail(MH_INVALID_ARG, "null argument or empty batch");
  if (n_inst > 4096) return fail(MH_UNSUPPORTED, "at most 4096 instances per batch");
  for (int i = 0; i < n_inst; ++i) {
    if (!meshes[i]) return fail(MH_INVALID_ARG, "null mesh");
    int rc = check_desc(&descs[i]);
    if (rc != MH_OK) return rc;
    const mh_op_desc& a = descs[0];
    const mh_op_desc& b = descs[i];
    if (a.n_orb != b.n_orb || a.n_alpha != b.n_alpha || a.n_beta != b.n_beta || a.lmax_bc != b.lmax_bc ||
        a.gauge != b.gauge)
      return fail(MH_INVALID_ARG, "instances of a batch must share n_orb, electron counts, lmax_bc and the gauge");
    if (meshes[i]->M.P != meshes[0]->M.P) return fail(MH_INVALID_ARG, "instances of a batch must share p");
  }
  return guarded([&]() -> int {
    std::vector<InstanceSpec> spec;
    for (int i = 0; i < n_inst; ++i) spec.push_back(make_spec(meshes[i], &descs[i], field_scale ? field_scale[i] : 1.0));
    *out = create_batch(spec, descs[0], S(stream));
    return MH_OK;
  });
}

extern "C" int mh_op_destroy(mh_op* op) {
  delete op;
  return MH_OK;
}

extern "C" int mh_op_sizes_get(const mh_op* op, mh_op_sizes* sz) {
  if (!op || !sz) return fail(MH_INVALID_ARG, "null argument");
  int64_t N = 0, nnz = 0;
  for (int i = 0; i < op->ni; ++i) {
    N += op->dh[i].N;
    nnz += (int64_t)op->Hs[i].kt_col.size();
  }
  sz->n_dof = N;
  sz->n_ext = op->B.tE;
  sz->n_full = op->B.tF;
  sz->n_ci = op->ci.dim;
  sz->n_orb = op->n;
  sz->n_pair_cols = op->ncol;
  sz->n_poisson_nnz = nnz;
  sz->n_inst = op->ni;
  return MH_OK;
}

extern "C" int mh_batch_layout(const mh_op* op, int64_t* layout) {
  if (!op || !layout) return fail(MH_INVALID_ARG, "null argument");
  for (int i = 0; i < op->ni; ++i) {
    const DevMesh& d = op->dh[i];
    int64_t* r = layout + 6 * (size_t)i;
    r[0] = d.N;
    r[1] = d.NE;
    r[2] = d.NF;
    r[3] = d.oE;
    r[4] = d.oF;
    r[5] = (int64_t)op->Hs[i].kt_col.size();
  }
  return MH_OK;
}

// ------------------------------------------------------- internal pieces ----
// Node-centric operator pass with optional event timing on the launch stream.
static void stencil_orb(mh_op* op, const double* u, const double* Ef, int diag_mode, int mode, double* out,
                        hipStream_t s) {
  const bool rec = op->timing && op->ev_used[0] + 2 <= (int)op->ev[0].size();
  if (rec) HIPCHK(hipEventRecord(op->ev[0][op->ev_used[0]], s));
  launch_stencil_orb(op->B, u, Ef, diag_mode, op->Upk, op->ginv, mode, op->lam, out, op->acc, op->kq, op->kred, s);
  if (rec) {
    HIPCHK(hipEventRecord(op->ev[0][op->ev_used[0] + 1], s));
    op->ev_used[0] += 2;
  }
}

// out = F(u) load vector over DoF rows (diag_mode 1: H1 only, 2: with mean
// field) at the field value held in the device scalar *Ef.
static void load_vector(mh_op* op, const double* u, const double* Ef, int diag_mode, double* out, hipStream_t s) {
  stencil_orb(op, u, Ef, diag_mode, 0, out, s);
  launch_ma_gather_orb(op->B, op->acc, 0, out, nullptr, s);
}

// out (extended) = G u  (or M^-1 F(u) when with_lam == 0)
static void g_apply(mh_op* op, const double* u, double* out, int with_lam, hipStream_t s) {
  const Batch& B = op->B;
  stencil_orb(op, u, op->Ebuf, 2, with_lam ? 2 : 1, out, s);
  launch_ma_gather_orb(B, op->acc, 1, out, op->ma_b, s);
  launch_ma_solve(B, op->ma_b, op->ma_x, op->ma_r, op->ma_d0, op->ma_d1, u, with_lam ? op->lam : nullptr, out, s);
  launch_fill_orb(B, out, nullptr, s);
}

// Poisson set-up of one solve: moments, boundary values, right-hand side, CG start.
static void poisson_begin(mh_op* op, const double* phi, double* W, int warm, hipStream_t s) {
  const Batch& B = op->B;
  PoissonWs& P = op->P;
  launch_poisson_pipeline_moments(B, phi, op->colinfo, P, s);
  launch_bnd_eval(B, P, W, s);
  launch_poisson_rhs_full(B, phi, W, op->colinfo, P.r, P, s);
  launch_cg_start(B, W, P.r, P, warm, s);
}

// 1 when every column of every instance meets the residual target, -1 on a
// non-finite residual, else 0 (reads the CG scalars after a stream sync).
// The target is relative to the largest right-hand side of the instance's
// columns, so a column whose right-hand side is rounding noise (the
// imaginary part of a real pair density) is held to the same absolute
// accuracy as the others; a warm start far from its solution could not reach
// a target relative to the noise itself.
static int poisson_converged(mh_op* op, hipStream_t s) {
  const int ncol = op->ncol, ni = op->ni;
  double* hs = op->hostpin;
  double* hr = hs + (size_t)ni * 8 * ncol;
  HIPCHK(hipMemcpyAsync(hs, op->P.sc, (size_t)ni * 8 * ncol * sizeof(double), hipMemcpyDeviceToHost, s));
  HIPCHK(hipMemcpyAsync(hr, op->P.red, (size_t)ni * RED_SLOTS * ncol * sizeof(double), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  const int rr_slot = op->P.it > 0 ? red_rr_slot(op->P.it) : -1;
  int conv = 1;
  for (int i = 0; i < ni; ++i) {
    const double* sc = hs + (size_t)i * 8 * ncol;
    const double* rd = hr + (size_t)i * RED_SLOTS * ncol;
    double bb = 0.0;
    for (int c = 0; c < ncol; ++c) bb = std::max(bb, sc[SC_BB * ncol + c]);
    for (int c = 0; c < ncol; ++c) {
      const double rr = rr_slot >= 0 ? rd[rr_slot * ncol + c] : sc[SC_RR * ncol + c];
      if (!std::isfinite(rr)) return -1;
      if (rr > op->rtol * op->rtol * bb) conv = 0;
    }
  }
  return conv;
}

// The multigrid hierarchies of all instances (Poisson schedule bit 4): host
// set-up of the coarse spaces, their operators and transfers (instances in
// parallel), then upload, the dense inverses of the coarsest operators on the
// device, and the per-level instance records.  Level 0 reuses
// each instance's assembled matrix and diagonal on the device, and its
// vectors live in batch arrays with the instances' extended-row offsets (the
// right-hand side is the CG residual itself).
static void ensure_mg(mh_op* op, hipStream_t s) {
  if (op->mg) return;
  const int ni = op->ni, ncol = op->ncol;
  // The coarsest level is solved by its dense inverse.  One instance takes
  // the first level with at most 2048 unknowns (one launch instead of the
  // smoothing and transfers of further levels, which cost more in launch
  // latency than the dense matrix costs in bytes); a batch stops at 400
  // unknowns, where the dense matrices of all instances are read every cycle.
  const int max_coarse = ni == 1 ? 2048 : 400;
  std::vector<MgHost> H(ni);
  {
    const int nthr = std::max(1, std::min<int>(ni, std::min(16u, std::max(1u, std::thread::hardware_concurrency()))));
    std::vector<std::thread> pool;
    std::vector<std::string> errs(nthr);
    for (int t = 0; t < nthr; ++t)
      pool.emplace_back([&, t]() {
        try {
          for (int i = t; i < ni; i += nthr) build_multigrid(op->Ms[i], op->Hs[i], H[i], max_coarse);
        } catch (const std::exception& e) {
          errs[t] = e.what();
        }
      });
    for (auto& th : pool) th.join();
    for (auto& e : errs)
      if (!e.empty()) throw std::runtime_error(e);
  }
  auto mg = std::make_unique<MgDev>();
  int nlev = 0;
  for (const MgHost& h : H) nlev = std::max(nlev, (int)h.lv.size());
  if (nlev < 1 || nlev > 32) throw std::runtime_error("multigrid hierarchy depth out of range");
  const size_t tlen = (size_t)op->B.tE * ncol;
  mg->z0 = op->alloc<double>(tlen);
  mg->z0b = op->alloc<double>(tlen);
  mg->t0 = op->alloc<double>(tlen);
  double* d0 = op->alloc<double>(tlen);
  mg->d0 = d0;
  HIPCHK(hipMemsetAsync(mg->z0, 0, tlen * sizeof(double), s));
  HIPCHK(hipMemsetAsync(mg->z0b, 0, tlen * sizeof(double), s));
  HIPCHK(hipMemsetAsync(mg->t0, 0, tlen * sizeof(double), s));
  HIPCHK(hipMemsetAsync(d0, 0, tlen * sizeof(double), s));
  // the same level-0 arrays on float storage (Poisson schedule bit 6)
  mg->z0f = op->alloc<float>(tlen);
  mg->z0bf = op->alloc<float>(tlen);
  mg->t0f = op->alloc<float>(tlen);
  mg->d0f = op->alloc<float>(tlen);
  mg->rf = op->alloc<float>(tlen);
  for (float* f : {mg->z0f, mg->z0bf, mg->t0f, mg->d0f, mg->rf}) HIPCHK(hipMemsetAsync(f, 0, tlen * sizeof(float), s));
  // level-0 Chebyshev coefficients of the fused smoothing passes: s0 = 1/theta
  // (first step), then c1, c2 of each later step of the three-term recurrence
  for (int i = 0; i < ni; ++i) {
    const double b = H[i].lv[0].lmax, a = b / MG_RANGE;
    const double theta = 0.5 * (b + a), delta = 0.5 * (b - a), sigma = theta / delta;
    double rho = 1.0 / sigma;
    op->dh[i].mgc[0] = 1.0 / theta;
    for (int k = 1; k < MG_MAX_DEG; ++k) {
      const double rn = 1.0 / (2.0 * sigma - rho);
      op->dh[i].mgc[2 * k - 1] = rn * rho;
      op->dh[i].mgc[2 * k] = 2.0 * rn / delta;
      rho = rn;
    }
  }
  // convergence flags of a batch's CG: every CG and multigrid launch of an
  // instance returns at once while its flag is set (batches only)
  if (ni > 1) {
    op->cg_done = op->alloc<int>(ni);
    HIPCHK(hipMemsetAsync(op->cg_done, 0, ni * sizeof(int), s));
    for (int i = 0; i < ni; ++i) op->dh[i].cg_done = op->cg_done + i;
  }
  upload_instances(op, s);
  std::vector<std::vector<MgLevelDev>> rec(nlev, std::vector<MgLevelDev>(ni));
  std::vector<MgLevelDev> co(ni);
  for (int i = 0; i < ni; ++i) {
    const DevMesh& dh = op->dh[i];
    const int nl = (int)H[i].lv.size();
    const size_t off = (size_t)dh.oE * ncol;
    for (int l = 0; l < nl; ++l) {
      const MgLevel& h = H[i].lv[l];
      MgLevelDev& L = rec[l][i];
      L.N = h.N;
      L.active = l + 1 < nl;
      L.coarse = l + 1 == nl;
      if (l == 0) {
        L.a_ptr = dh.kt_ptr;
        L.a_col = dh.kt_col;
        L.a_val = dh.kt_val;
        L.dinv = dh.kdiag_inv;
        L.r = op->P.r + off;
        L.z = mg->z0 + off;
        L.t = mg->t0 + off;
        L.d = d0 + off;
        L.rf = mg->rf + off;
        L.zf = mg->z0f + off;
        L.tf = mg->t0f + off;
      } else {
        L.a_ptr = op->upload(h.k_ptr, s);
        L.a_col = op->upload(h.k_col, s);
        L.a_val = op->upload(h.k_val, s);
        L.dinv = op->upload(h.dinv, s);
        const size_t len = (size_t)std::max<int64_t>(1, h.N) * ncol;
        L.r = op->alloc<double>(len);
        L.z = op->alloc<double>(len);
        L.d = op->alloc<double>(len);
        L.t = op->alloc<double>(len);
      }
      L.lmax = h.lmax;
      L.done = op->cg_done ? op->cg_done + i : nullptr;
      if (L.active) {
        L.p_ptr = op->upload(h.p_ptr, s);
        L.p_col = op->upload(h.p_col, s);
        L.p_val = op->upload(h.p_val, s);
        L.r_ptr = op->upload(h.r_ptr, s);
        L.r_col = op->upload(h.r_col, s);
        L.r_val = op->upload(h.r_val, s);
      } else {
        double* ci = op->upload(H[i].coarse_dense, s);
        launch_dense_inverse(ci, h.N, s);  // Gauss-Jordan (the operator is SPD)
        L.cinv = ci;
        co[i] = L;
        mg->max_coarse = std::max(mg->max_coarse, h.N);
      }
      mg->max_n[l] = std::max(mg->max_n[l], h.N);
    }
  }
  mg->nlev = nlev;
  for (int l = 0; l < nlev; ++l) mg->lv.push_back(op->upload(rec[l], s));
  mg->lv0_double = mg->lv[0];
  for (MgLevelDev& L : rec[0]) L.f32 = 1;
  mg->lv0_float = op->upload(rec[0], s);
  mg->coarse = op->upload(co, s);
  op->mg_red = op->alloc<double>((size_t)ni * RED_SLOTS * ncol);
  op->mg_part = op->alloc<double>((size_t)ni * MG_RZ_BLOCKS * ncol);
  HIPCHK(hipStreamSynchronize(s));  // the host tables are temporaries
  op->mg_levels = nlev;
  op->mg = std::move(mg);
}

// CG preconditioned by one multigrid V-cycle per instance and iteration,
// after launch_cg_start (r_0 in P.r, accumulators initialised): z = B r,
// rz = r.z, p = z + beta p, then the same operator and update passes as the
// Jacobi CG (alpha = r.z / p.q), with every instance's own scalars.  With a
// smoothed finest level, r.z is accumulated by the cycle's last smoothing
// pass; else it takes passes of its own.
// Converged (1), not (0) or non-finite (-1).  The check (a host round trip)
// runs before the first iteration and after every iteration from two before
// the previous solve's count on (successive solves of a propagation take
// nearly the same count; an unchecked iteration only lowers the residual).
// fixed > 0: exactly `fixed` iterations with no host check (the launch
// sequence of a captured step; every update stays well defined past
// convergence, alpha and beta being zero where their denominators vanish);
// the caller checks the residual afterwards.
static int mg_pcg(mh_op* op, double* W, int* iters, hipStream_t s, int fixed = 0) {
  const Batch& B = op->B;
  PoissonWs& P = op->P;
  const MgDev& mg = *op->mg;
  const int ncol = op->ncol, ni = op->ni;
  const int64_t N = B.mx.N;
  // Poisson schedule bits 8-9: Chebyshev smoothing degree 2 + their value
  op->mg->nu = 2 + ((B.mx.sched_poi >> 8) & 3);
  const int nu = mg.nu;
  const bool fused = mg.nlev > 1 && nu >= 2;
  // Poisson schedule bit 6: the finest level's smoothing passes, residual
  // pass and transfers on float copies of its arrays (the preconditioner
  // only; the CG vectors, its operator pass and every sum stay double)
  const bool f32 = fused && (B.mx.sched_poi & 64);
  op->mg->lv[0] = f32 ? mg.lv0_float : mg.lv0_double;
  int rz_slot = RED_RZ;
  // the level-0 correction alternates between two buffers (a smoothing step
  // reads one and writes the other): zc = 1 while it is in the second.  The
  // pre-smoothing starts in the buffer that makes it end in the first, where
  // the residual pass and the prolongation read it; after the post-smoothing
  // it ends in the second when the degree is odd.
  int zc = 0;
  MgLevel0Ops ops;
  if (f32) {
    ops.resid = [&](hipStream_t st) { launch_mg_resid_f(B, mg.z0f, mg.rf, mg.t0f, ncol, op->mg_red, st); };
    ops.cheb0 = [&](hipStream_t st) {
      zc = nu % 2;
      launch_mg_cheb0_f(B, mg.rf, zc ? mg.z0bf : mg.z0f, mg.d0f, P.red, rz_slot | (nu > 2 ? 0 : 256), ncol, st);
    };
    ops.cheb = [&](int k, bool rz, hipStream_t st) {
      float* zi = zc ? mg.z0bf : mg.z0f;
      float* zo = zc ? mg.z0f : mg.z0bf;
      zc ^= 1;
      launch_mg_cheb_step_f(B, zi, mg.rf, zo, mg.d0f, P.red, ncol, k, rz ? rz_slot : -1, st);
    };
  } else {
    ops.resid = [&](hipStream_t st) { launch_mg_resid(B, mg.z0, P.r, mg.t0, ncol, op->mg_red, st); };
    ops.cheb0 = [&](hipStream_t st) {
      zc = nu % 2;
      launch_mg_cheb0(B, P.r, zc ? mg.z0b : mg.z0, mg.d0, P.red, rz_slot | (nu > 2 ? 0 : 256), ncol, st);
    };
    ops.cheb = [&](int k, bool rz, hipStream_t st) {
      double* zi = zc ? mg.z0b : mg.z0;
      double* zo = zc ? mg.z0 : mg.z0b;
      zc ^= 1;
      launch_mg_cheb_step(B, zi, P.r, zo, mg.d0, P.red, ncol, k, rz ? rz_slot : -1, st);
    };
  }
  // the preconditioned residual after a fused cycle (single level: the dense solve's z0)
  double* z = fused && nu % 2 ? mg.z0b : mg.z0;
  float* zf = nu % 2 ? mg.z0bf : mg.z0f;
  auto precondition = [&](int it) {  // z = B r with r.z in slot RED_RZ + it % 3
    rz_slot = RED_RZ + it % 3;
    mg_vcycle(mg, ni, ncol, ops, s);
    if (!fused) mg_rz(B.dm, ni, ncol, P.r, z, op->mg_part, P.red, rz_slot, s);
  };
  P.it = 0;
  if (op->cg_done) launch_zero_int(op->cg_done, ni, s);  // batch convergence flags start clear
  int conv = fixed > 0 ? 0 : poisson_converged(op, s);
  int k = 0;
  const int check_from = op->cg_hint - 2;
  const int kmax = fixed > 0 ? fixed : op->maxit;
  if (conv == 0) {
    if (f32) launch_to_float(P.r, mg.rf, (int64_t)B.tE * ncol, s);  // later residuals by the update pass
    precondition(0);
  }
  // one instance: each iteration's x += alpha p is deferred to the next
  // direction pass, which reads p anyway (and to cg_xfinal after the last);
  // a batch keeps it in the update pass (its instances stop at different
  // iterations)
  const bool defer = ni == 1;
  double* xd = defer ? W : nullptr;
  while (conv == 0 && k < kmax) {
    double* pcur = (k % 2) ? P.p2 : P.p;
    double* pold = (k % 2) ? P.p : P.p2;
    const int pq_prev = RED_PQ + (k + 1) % 2;   // the p.q slot of iteration k - 1
    if (f32)
      mg_dir(B.dm, ni, N, ncol, zf, pold, pcur, P.red, RED_RZ + k % 3, k > 0 ? RED_RZ + (k - 1) % 3 : -1,
             RED_RR + k % 2, xd, pq_prev, s);
    else
      mg_dir(B.dm, ni, N, ncol, z, pold, pcur, P.red, RED_RZ + k % 3, k > 0 ? RED_RZ + (k - 1) % 3 : -1,
             RED_RR + k % 2, xd, pq_prev, s);
    launch_cg_apply_plain(B, P, pcur, k, s);
    launch_cg_update(B, W, P, pcur, k, s, f32 ? mg.rf : nullptr, defer ? 0 : 1);
    if (op->cg_done) launch_cg_done(B, P, k, op->rtol, s);  // converged instances skip the rest
    ++k;
    P.it = k;
    if (fixed > 0) {
      if (k < fixed) precondition(k);
      continue;
    }
    if (k >= check_from || k == op->maxit) conv = poisson_converged(op, s);
    if (conv != 0) break;
    precondition(k);
  }
  if (defer && k > 0)   // the last iteration's x += alpha p
    cg_xfinal(B.dm, ni, N, ncol, W, ((k - 1) % 2) ? P.p2 : P.p, P.red, RED_RZ + (k - 1) % 3, RED_PQ + (k - 1) % 2, s);
  if (op->cg_done) launch_zero_int(op->cg_done, ni, s);  // no flag outside the CG
  if (iters) *iters = k;
  if (fixed == 0) op->cg_hint = k;
  return conv;
}

// CG iterations after launch_cg_start, to the residual target or the cap:
// multigrid-preconditioned (Poisson schedule bit 4), else
// Jacobi launch by launch with a convergence check every 8 iterations.
// 1 converged, 0 not, -1 non-finite residual.
static int cg_iterate(mh_op* op, double* W, int* iters, hipStream_t s) {
  const Batch& B = op->B;
  PoissonWs& P = op->P;
  if (B.mx.sched_poi & 16) {
    ensure_mg(op, s);
    return mg_pcg(op, W, iters, s);
  }
  int it = 0, conv = 0;
  const int check = 8;
  while (it < op->maxit) {
    int todo = std::min(check, op->maxit - it);
    for (int k = 0; k < todo; ++k) launch_cg_step(B, W, P, s);
    it += todo;
    conv = poisson_converged(op, s);
    if (conv != 0) break;
  }
  if (iters) *iters = it;
  return conv;
}

static int poisson_solve(mh_op* op, const double* phi, double* W, int warm, int* iters, hipStream_t s) {
  const Batch& B = op->B;
  PoissonWs& P = op->P;
  poisson_begin(op, phi, W, warm, s);
  const int conv = cg_iterate(op, W, iters, s);
  if (conv < 0) return fail(MH_NONFINITE, "non-finite Poisson residual");
  launch_fill_real(B, W, 1, op->ncol, 1, P.acc, s);
  return conv ? MH_OK : MH_NOT_CONVERGED;
}

// Frozen data of G at the current orbitals (field value already in Ebuf[0]):
// U from W and Gamma, gamma^-1, lambda = c^H F(c).
static void freeze_body(mh_op* op, const double* phi, const double* gamma, const double* Gamma, const double* W,
                        hipStream_t s) {
  const Batch& B = op->B;
  launch_build_U_full(B, W, Gamma, op->colmap, op->Mr, op->Upk, s);
  launch_ginv(op->ni, gamma, op->n, op->rdm_eps, op->ginv, op->flag, s);
  load_vector(op, phi, op->Ebuf, 2, op->F, s);
  launch_gram(B, phi, op->F, WT_NONE, ROWS_DOF, op->gpart, gram_blocks(B.mx.N), op->lam, s);
  op->frozen = true;
}

static int freeze(mh_op* op, const double* phi, const double* gamma, const double* Gamma, double E, const double* W,
                  hipStream_t s) {
  launch_set(op->Ebuf, E, s);
  freeze_body(op, phi, gamma, Gamma, W, s);
  return MH_OK;
}

static void ensure_krylov(mh_op* op, int m) {
  if (op->m_alloc >= m) return;
  for (double* p : op->V) {
    op->release(p);
  }
  op->V.clear();
  const size_t len = (size_t)2 * op->B.tE * op->n;
  for (int j = 0; j <= m; ++j) op->V.push_back(op->alloc<double>(len));
  op->Vdev = op->alloc<double*>(m + 1);
  HIPCHK(hipMemcpy(op->Vdev, op->V.data(), (m + 1) * sizeof(double*), hipMemcpyHostToDevice));
  // enough workgroups to keep the memory system busy (the dot and update passes
  // stream whole vectors), about 8192 over a batch (grid.y = instance)
  int64_t nb = std::min<int64_t>(2048, std::max<int64_t>(1, (op->B.mx.NE * op->n + 255) / 256));
  if (op->ni > 1) nb = std::min<int64_t>(nb, std::max<int64_t>(8, 8192 / op->ni));
  const int nblk = (int)nb;
  krylov_alloc(op, op->K, m, nblk);
  op->m_alloc = m;
}

// With an error threshold (krylov_tol > 0) the space stops growing at the
// first dimension whose error estimate meets it (Sec. III.B), m being the
// largest: after each vector the estimate is evaluated on the device and the
// instances' dimensions read back (one small synchronising read per vector);
// a batch grows until every instance has stopped.
static int arnoldi(mh_op* op, double* phi, double tau_re, double tau_im, int m, hipStream_t s) {
  const Batch& B = op->B;
  ensure_krylov(op, m);
  Krylov K = op->K;
  K.m_max = op->m_alloc;
  launch_norm_init(B, phi, K, m, s);
  launch_krylov_scale(B, phi, op->V[0], K, 5, s);
  const bool adaptive = op->krylov_tol > 0.0;
  int built = m;
  for (int k = 0; k < m; ++k) {
    double* w = op->V[k + 1];
    g_apply(op, op->V[k], w, 1, s);
    launch_mdot(B, op->Vdev, k, w, K, 1, s);
    launch_orth_dot(B, op->Vdev, k, w, K, s);
    launch_orth_update(B, op->Vdev, k, w, K, 2, s);
    launch_krylov_scale(B, w, w, K, 1, s);
    if (adaptive && k + 1 < m) {
      launch_krylov_check(op->ni, K, tau_re, tau_im, k + 1, op->krylov_tol, s);
      HIPCHK(hipMemcpyAsync(op->hostpin, K.scal, (size_t)op->ni * 8 * sizeof(double), hipMemcpyDeviceToHost, s));
      HIPCHK(hipStreamSynchronize(s));
      bool all = true;
      for (int i = 0; i < op->ni; ++i)
        if ((int)op->hostpin[8 * i + 4] > k + 1) all = false;
      if (all) {
        built = k + 1;
        break;
      }
    }
  }
  launch_expm(op->ni, K, tau_re, tau_im, s);
  launch_combine(B, op->Vdev, built, phi, K, s);
  return MH_OK;
}

// ------------------------------------------------------------ entry points ----
extern "C" int mh_fill_hanging(mh_op* op, double* x, void* stream) {
  if (!op || !x) return fail(MH_INVALID_ARG, "null argument");
  return guarded([&]() -> int {
    launch_fill_orb(op->B, x, nullptr, S(stream));
    HIPCHK(hipGetLastError());
    return MH_OK;
  });
}

extern "C" int mh_mass_solve(mh_op* op, const double* f, double* c, void* stream) {
  if (!op || !f || !c) return fail(MH_INVALID_ARG, "null argument");
  return guarded([&]() -> int {
    hipStream_t s = S(stream);
    const Batch& B = op->B;
    launch_mass_direct(B, f, c, op->ma_b, s);
    launch_ma_solve(B, op->ma_b, op->ma_x, op->ma_r, op->ma_d0, op->ma_d1, nullptr, nullptr, c, s);
    launch_fill_orb(B, c, nullptr, s);
    HIPCHK(hipGetLastError());
    return MH_OK;
  });
}

extern "C" int mh_mass_solve_noalloc(mh_op* op, const double* f, double* c, void* stream) {
  if (!op || !f || !c) return fail(MH_INVALID_ARG, "null argument");
  return guarded([&]() -> int {
    hipStream_t s = S(stream);
    const Batch& B = op->B;
    // five buffers of [sum of interface unknowns][n] complex values
    const size_t buf = 2 * std::max<size_t>(1, B.tMa) * (size_t)op->n;   // doubles per buffer
    const size_t need = 5 * buf * sizeof(double);
    if (need > kScratchBytes)
      return fail(MH_UNSUPPORTED, "interface mass system needs " + std::to_string(need) + " bytes of scratch, more than the " +
                                      std::to_string(kScratchBytes) + " bytes of mh_mass_solve_noalloc");
    int dev = 0;
    HIPCHK(hipGetDevice(&dev));
    if (dev != op->device) return fail(MH_INVALID_ARG, "call on the device the operator was created on");
    double* base = static_cast<double*>(scratch_on(dev));
    if (!base) return fail(MH_INVALID_ARG, "scratch of this device not set up");
    // every scratch element the kernels read is written first in this call
    // (gather of the right-hand side, then the iteration's initial state)
    double* mb = base;
    launch_mass_direct(B, f, c, mb, s);
    launch_ma_solve(B, mb, mb + buf, mb + 2 * buf, mb + 3 * buf, mb + 4 * buf, nullptr, nullptr, c, s);
    launch_fill_orb(B, c, nullptr, s);
    HIPCHK(hipGetLastError());
    return MH_OK;
  });
}

extern "C" int mh_h1_apply(mh_op* op, const double* c, double E, double* f, void* stream) {
  if (!op || !c || !f) return fail(MH_INVALID_ARG, "null argument");
  return guarded([&]() -> int {
    hipStream_t s = S(stream);
    launch_set(op->Ebuf + 1, E, s);
    load_vector(op, c, op->Ebuf + 1, 1, f, s);
    HIPCHK(hipGetLastError());
    return MH_OK;
  });
}

extern "C" int mh_poisson_pairs(mh_op* op, const double* phi, double* W, int32_t warm, int32_t* iters,
                                void* stream) {
  if (!op || !phi || !W) return fail(MH_INVALID_ARG, "null argument");
  return guarded([&]() -> int {
    int it = 0;
    int rc = poisson_solve(op, phi, W, warm, &it, S(stream));
    HIPCHK(hipStreamSynchronize(S(stream)));
    if (iters) *iters = it;
    if (rc == MH_NOT_CONVERGED) g_err = "Poisson CG reached poisson_maxit";
    return rc;
  });
}

extern "C" int mh_ci_rdms(mh_op* op, const double* Ci, double* gamma, double* Gamma, void* stream) {
  if (!op || !Ci || !gamma || !Gamma) return fail(MH_INVALID_ARG, "null argument");
  return guarded([&]() -> int {
    launch_ci_rdm_full(op->ni, op->ci, Ci, gamma, Gamma, op->Gtmp, S(stream));
    HIPCHK(hipGetLastError());
    return MH_OK;
  });
}

static bool any_flag(mh_op* op, hipStream_t s) {
  int* hf = (int*)op->hostpin;
  HIPCHK(hipMemcpyAsync(hf, op->flag, op->ni * sizeof(int), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  for (int i = 0; i < op->ni; ++i)
    if (hf[i]) return true;
  return false;
}

extern "C" int mh_freeze(mh_op* op, const double* phi, const double* gamma, const double* Gamma, double E,
                         const double* W, void* stream) {
  if (!op || !phi || !gamma || !Gamma || !W) return fail(MH_INVALID_ARG, "null argument");
  return guarded([&]() -> int {
    hipStream_t s = S(stream);
    freeze(op, phi, gamma, Gamma, E, W, s);
    if (any_flag(op, s)) {
      op->frozen = false;
      return fail(MH_SINGULAR_RDM, "1-RDM not positive after regularisation");
    }
    return MH_OK;
  });
}

extern "C" int mh_rhs_apply(mh_op* op, const double* v, double* Gv, void* stream) {
  if (!op || !v || !Gv) return fail(MH_INVALID_ARG, "null argument");
  if (!op->frozen) return fail(MH_INVALID_ARG, "mh_freeze has not been called");
  return guarded([&]() -> int {
    g_apply(op, v, Gv, 1, S(stream));
    HIPCHK(hipGetLastError());
    return MH_OK;
  });
}

extern "C" int mh_arnoldi_step(mh_op* op, double* phi, double tau_re, double tau_im, int32_t m, double* err_est,
                               int32_t* m_used, void* stream) {
  if (!op || !phi) return fail(MH_INVALID_ARG, "null argument");
  if (m < 1 || m > 24) return fail(MH_INVALID_ARG, "Krylov dimension must be 1..24");
  if (!op->frozen) return fail(MH_INVALID_ARG, "mh_freeze has not been called");
  return guarded([&]() -> int {
    hipStream_t s = S(stream);
    arnoldi(op, phi, tau_re, tau_im, m, s);
    HIPCHK(hipGetLastError());
    if (err_est || m_used) {
      HIPCHK(hipMemcpyAsync(op->hostpin, op->K.scal, (size_t)op->ni * 8 * sizeof(double), hipMemcpyDeviceToHost, s));
      HIPCHK(hipStreamSynchronize(s));
      double err = 0.0;
      int mu = m;
      for (int i = 0; i < op->ni; ++i) {
        err = std::max(err, op->hostpin[8 * i + 3]);
        mu = std::min(mu, (int)op->hostpin[8 * i + 4]);
      }
      if (err_est) *err_est = err;
      if (m_used) *m_used = mu;
    }
    return MH_OK;
  });
}

// Everything of one time step after the Poisson solve, with the step's field
// value already in Ebuf[0]: freeze, one- and two-electron integrals and
// observables at t_n, then (advance) the orbital Arnoldi step and the CI
// Lanczos step.  A fixed launch sequence, so it can be captured as a graph.
static void step_after_poisson(mh_op* op, double* phi, double* Ci, const double* W, int advance, double tre,
                               double tim, int m, int imaginary, hipStream_t s) {
  const Batch& B = op->B;
  const int mci = std::min(12, op->ci.dim);
  freeze_body(op, phi, op->gam, op->Gam, W, s);
  load_vector(op, phi, op->Ebuf, 1, op->F, s);
  launch_gram(B, phi, op->F, WT_NONE, ROWS_DOF, op->gpart, gram_blocks(B.mx.N), op->hmat, s);
  launch_gint_full(B, phi, W, op->colmap, op->gpart, gint_blocks(B), op->Gtmp, op->gint, s);
  launch_gram(B, phi, phi, WT_MASS, ROWS_EXT, op->gpart, gram_blocks(B.mx.NE), op->S, s);
  launch_gram(B, phi, phi, WT_DIPOLE, ROWS_EXT, op->gpart, gram_blocks(B.mx.NE), op->zmat, s);
  load_vector(op, phi, op->Ebuf, 4, op->F, s);   // -i S_e phi: momentum along e
  launch_gram(B, phi, op->F, WT_NONE, ROWS_DOF, op->gpart, gram_blocks(B.mx.N), op->pmat, s);
  launch_observe(B, op->gam, op->Gam, op->hmat, op->gint, op->zmat, op->S, op->pmat, op->Ebuf, op->obs, s);
  if (!advance) return;
  arnoldi(op, phi, tre, tim, m, s);
  launch_ci_hprime(op->ni, op->ci, op->hmat, op->gint, s);
  launch_ci_lanczos(op->ni, op->ci, op->Qdev, op->Qh.data(), mci, op->gint, Ci, op->KC, tre, tim, imaginary ? 1 : 0,
                    s);
  if (imaginary) {
    launch_gram(B, phi, phi, WT_MASS, ROWS_EXT, op->gpart, gram_blocks(B.mx.NE), op->S, s);
    launch_orthonormalize_full(B, op->S, op->Rinv, phi, s);
  }
}

namespace {
// One whole time step as a fixed launch sequence (MH_PROP_GRAPH_STEP), for
// the steps whose CG start is the quadratic extrapolation: the RDMs, the
// start, the pair Poisson solves with `K` multigrid-preconditioned CG
// iterations and no host check, the boundary fill, the step's field value
// from the device table, then the step after the Poisson solve; the counter
// moves on to the next step.
static void whole_step(mh_op* op, double* phi, double* Ci, double* W, int K, double tre, double tim, int m,
                       int imaginary, hipStream_t s) {
  const Batch& B = op->B;
  const int64_t wlen = (int64_t)B.tF * op->ncol;
  launch_ci_rdm_full(op->ni, op->ci, Ci, op->gam, op->Gam, op->Gtmp, s);
  launch_extrapolate2(W, op->Wprev, op->Wprev2, wlen, s);
  poisson_begin(op, phi, W, 1, s);
  mg_pcg(op, W, nullptr, s, K);
  launch_fill_real(B, W, 1, op->ncol, 1, op->P.acc, s);
  launch_set_indexed(op->Ebuf, op->Etab, op->step_ctr, s);
  step_after_poisson(op, phi, Ci, W, 1, tre, tim, m, imaginary, s);
  launch_counter(op->step_ctr, 0, 1, s);
}

// Copy the step's scalars to the host (a synchronising read) and file its
// records; MH_SINGULAR_RDM / MH_NONFINITE where the step went wrong.
static int record_step(mh_op* op, mh_observables* obs, int step, int advance, int it, hipStream_t s) {
  const int ni = op->ni;
  double* hs = op->hostpin;
  double* hk = hs + 8 * (size_t)ni;
  int* hf = (int*)(hs + 16 * (size_t)ni);
  HIPCHK(hipMemcpyAsync(hs, op->obs, (size_t)ni * 8 * sizeof(double), hipMemcpyDeviceToHost, s));
  if (advance) HIPCHK(hipMemcpyAsync(hk, op->K.scal, (size_t)ni * 8 * sizeof(double), hipMemcpyDeviceToHost, s));
  HIPCHK(hipMemcpyAsync(hf, op->flag, ni * sizeof(int), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  for (int i = 0; i < ni; ++i) {
    if (hf[i]) return fail(MH_SINGULAR_RDM, "1-RDM not positive after regularisation");
    if (!std::isfinite(hs[8 * i]) || !std::isfinite(hs[8 * i + 1])) return fail(MH_NONFINITE, "non-finite observables");
  }
  if (obs) {
    for (int i = 0; i < ni; ++i) {
      const size_t o = (size_t)step * ni + i;
      if (obs->dipole) obs->dipole[o] = hs[8 * i + 1];
      if (obs->energy) obs->energy[o] = hs[8 * i];
      if (obs->ortho) obs->ortho[o] = hs[8 * i + 2];
      if (obs->momentum) obs->momentum[o] = hs[8 * i + 3];
      if (obs->krylov_dim) obs->krylov_dim[o] = advance ? (int32_t)hk[8 * i + 4] : 0;
      if (obs->err_est) obs->err_est[o] = advance ? hk[8 * i + 3] : 0.0;
    }
    if (obs->cg_iters) obs->cg_iters[step] = it;
  }
  return MH_OK;
}

struct GraphHolder {
  hipGraph_t g = nullptr;
  hipGraphExec_t x = nullptr;
  ~GraphHolder() {
    if (x) (void)hipGraphExecDestroy(x);
    if (g) (void)hipGraphDestroy(g);
  }
};
struct EventHolder {
  hipEvent_t e[2] = {nullptr, nullptr};
  ~EventHolder() {
    for (hipEvent_t v : e)
      if (v) (void)hipEventDestroy(v);
  }
};
}  // namespace

extern "C" int mh_propagate(mh_op* op, double* phi, double* Ci, double* W, const double* E_steps, int32_t n_steps,
                            double dt, int32_t m, int32_t flags, mh_observables* obs, void* stream) {
  const int imaginary = flags & MH_PROP_IMAGINARY;
  const bool use_graph = (flags & MH_PROP_GRAPH) != 0;
  const bool graph_step = (flags & MH_PROP_GRAPH_STEP) != 0;
  const int last_step = (flags & MH_PROP_NO_FINAL) ? n_steps - 1 : n_steps;
  if (!op || !phi || !Ci || !W || (n_steps > 0 && !E_steps)) return fail(MH_INVALID_ARG, "null argument");
  if (n_steps < 0 || m < 1 || m > 24) return fail(MH_INVALID_ARG, "bad step count or Krylov dimension");
  if ((use_graph || graph_step) && op->krylov_tol > 0.0)
    return fail(MH_INVALID_ARG, "graph replay needs a fixed Krylov dimension (krylov_tol = 0)");
  if (use_graph && graph_step) return fail(MH_INVALID_ARG, "MH_PROP_GRAPH and MH_PROP_GRAPH_STEP exclude each other");
  if (graph_step && !(op->B.mx.sched_poi & 16))
    return fail(MH_INVALID_ARG, "whole-step graph replay needs the multigrid Poisson schedule (bit 4)");
  return guarded([&]() -> int {
    hipStream_t s = S(stream);
    const int ni = op->ni;
    const double tre = imaginary ? 0.0 : dt, tim = imaginary ? -dt : 0.0;
    int status = MH_OK;
    GraphHolder gh;
    EventHolder evh;
    const bool saved_timing = op->timing;
    if (use_graph || graph_step) {
      ensure_krylov(op, m);
      if (!op->gstream) HIPCHK(hipStreamCreateWithFlags(&op->gstream, hipStreamNonBlocking));
      HIPCHK(hipEventCreateWithFlags(&evh.e[0], hipEventDisableTiming));
      HIPCHK(hipEventCreateWithFlags(&evh.e[1], hipEventDisableTiming));
    }
    if (graph_step && n_steps > 3) {
      if (op->Etab_len < n_steps + 1) {
        op->Etab = op->alloc<double>((size_t)n_steps + 1);
        op->Etab_len = n_steps + 1;
      }
      if (!op->step_ctr) op->step_ctr = op->alloc<int>(1);
      HIPCHK(hipMemcpyAsync(op->Etab, E_steps, (size_t)(n_steps + 1) * sizeof(double), hipMemcpyHostToDevice, s));
      HIPCHK(hipStreamSynchronize(s));
      ensure_mg(op, s);
    }
    int K_fixed = 0;   // CG iterations of the replayed steps
    for (int step = 0; step <= last_step; ++step) {
      const double E = (n_steps > 0 || E_steps) ? E_steps[step] : 0.0;
      if (graph_step && step >= 3 && step < n_steps) {
        // whole step from the graph: one launch; then the residual check and
        // the step's records
        hipStream_t g = op->gstream;
        if (!gh.x) {
          K_fixed = op->cg_hint + 3;
          launch_counter(op->step_ctr, 1, step, s);
          op->timing = false;  // no timing events inside the graph
          hipEvent_t* saved_ev = op->P.ev;
          op->P.ev = nullptr;
          HIPCHK(hipEventRecord(evh.e[0], s));
          HIPCHK(hipStreamWaitEvent(g, evh.e[0], 0));
          HIPCHK(hipStreamBeginCapture(g, hipStreamCaptureModeThreadLocal));
          whole_step(op, phi, Ci, W, K_fixed, tre, tim, m, imaginary, g);
          HIPCHK(hipStreamEndCapture(g, &gh.g));
          HIPCHK(hipGraphInstantiate(&gh.x, gh.g, nullptr, nullptr, 0));
          op->P.ev = saved_ev;
          op->timing = saved_timing;
        }
        HIPCHK(hipEventRecord(evh.e[0], s));
        HIPCHK(hipStreamWaitEvent(g, evh.e[0], 0));
        HIPCHK(hipGraphLaunch(gh.x, g));
        HIPCHK(hipEventRecord(evh.e[1], g));
        HIPCHK(hipStreamWaitEvent(s, evh.e[1], 0));
        op->P.it = K_fixed;
        const int conv = poisson_converged(op, s);
        if (conv < 0) return fail(MH_NONFINITE, "non-finite Poisson residual");
        if (conv == 0) status = MH_NOT_CONVERGED;
        const int rr = record_step(op, obs, step, 1, K_fixed, s);
        if (rr != MH_OK) return rr;
        continue;
      }
      launch_ci_rdm_full(ni, op->ci, Ci, op->gam, op->Gam, op->Gtmp, s);
      int it = 0;
      // CG start: the previous solution; at the third step of the call the
      // linear extrapolation 2 W_{n-1} - W_{n-2}, from the fourth the quadratic
      // 3 W_{n-1} - 3 W_{n-2} + W_{n-3} (Wprev, Wprev2 keep W_{n-2}, W_{n-3})
      const int64_t wlen = (int64_t)op->B.tF * op->ncol;
      if (step == 0 && !op->Wprev) op->Wprev = op->alloc<double>((size_t)wlen);
      if (step == 0 && !op->Wprev2) op->Wprev2 = op->alloc<double>((size_t)wlen);
      if (step == 2) {
        launch_copy(op->Wprev, op->Wprev2, wlen, s);
        launch_extrapolate(W, op->Wprev, wlen, s);
      } else if (step >= 3) {
        launch_extrapolate2(W, op->Wprev, op->Wprev2, wlen, s);
      }
      int rc = poisson_solve(op, phi, W, 1, &it, s);
      if (step == 0) launch_copy(W, op->Wprev, wlen, s);  // W_0; step 1 starts from W_0 and keeps it
      if (rc < 0) return rc;
      if (rc == MH_NOT_CONVERGED) status = MH_NOT_CONVERGED;
      launch_set(op->Ebuf, E, s);
      const int advance = step < n_steps;
      if (use_graph && advance) {
        hipStream_t g = op->gstream;
        if (!gh.x) {
          op->timing = false;
          HIPCHK(hipEventRecord(evh.e[0], s));
          HIPCHK(hipStreamWaitEvent(g, evh.e[0], 0));
          HIPCHK(hipStreamBeginCapture(g, hipStreamCaptureModeThreadLocal));
          step_after_poisson(op, phi, Ci, W, 1, tre, tim, m, imaginary, g);
          HIPCHK(hipStreamEndCapture(g, &gh.g));
          HIPCHK(hipGraphInstantiate(&gh.x, gh.g, nullptr, nullptr, 0));
          op->timing = saved_timing;
        }
        HIPCHK(hipEventRecord(evh.e[0], s));
        HIPCHK(hipStreamWaitEvent(g, evh.e[0], 0));
        HIPCHK(hipGraphLaunch(gh.x, g));
        HIPCHK(hipEventRecord(evh.e[1], g));
        HIPCHK(hipStreamWaitEvent(s, evh.e[1], 0));
      } else {
        step_after_poisson(op, phi, Ci, W, advance, tre, tim, m, imaginary, s);
      }
      const int rr = record_step(op, obs, step, advance, it, s);
      if (rr != MH_OK) return rr;
    }
    return status;
  });
}

extern "C" int mh_kernel_timing(mh_op* op, int32_t which, int32_t enable, double* avg_ms, int64_t* count) {
  if (!op || which < 0 || which > 1) return fail(MH_INVALID_ARG, "bad argument");
  return guarded([&]() -> int {
    HIPCHK(hipDeviceSynchronize());
    const int cap = 8192;
    for (int k = 0; k < 2; ++k)
      while ((int)op->ev[k].size() < cap) {
        hipEvent_t e;
        HIPCHK(hipEventCreate(&e));
        op->ev[k].push_back(e);
      }
    op->ev_used[1] = op->P.ev_used;
    double tot = 0.0;
    int64_t cnt = 0;
    for (int i = 0; i + 1 < op->ev_used[which]; i += 2) {
      float ms = 0.f;
      HIPCHK(hipEventElapsedTime(&ms, op->ev[which][i], op->ev[which][i + 1]));
      tot += ms;
      ++cnt;
    }
    if (avg_ms) *avg_ms = cnt ? tot / cnt : 0.0;
    if (count) *count = cnt;
    op->ev_used[which] = 0;
    if (which == 1) op->P.ev_used = 0;
    op->timing = enable != 0;
    op->P.ev = op->timing ? op->ev[1].data() : nullptr;
    op->P.ev_cap = cap;
    return MH_OK;
  });
}

// Sliced-ELL copy of the short rows of an instance's assembled Poisson
// operator: within each window of SELL_WINDOW rows the short rows are sorted
// by length (longest first, stable) and cut into slices of SELL_H slots; a
// slice is as wide as its longest row, rounded up to a multiple of 4, and its
// entries are stored slot-fastest so that the lanes of a wave, one row each,
// read consecutive words.  Padding entries repeat the slot's own row as the
// column (empty slots: row 0) with coefficient 0.
static void build_sell(mh_op* op, int i, hipStream_t s) {
  DevMesh& d = op->dh[i];
  const OpHost& H = op->Hs[i];
  const int64_t N = d.N;
  std::vector<int32_t> ptr{0}, row, col;
  std::vector<double> val;
  std::vector<int32_t> win;
  for (int64_t w0 = 0; w0 < N; w0 += SELL_WINDOW) {
    win.clear();
    const int64_t w1 = std::min<int64_t>(N, w0 + SELL_WINDOW);
    for (int64_t r = w0; r < w1; ++r)
      if (H.kt_ptr[r + 1] - H.kt_ptr[r] <= KT_LONG) win.push_back((int32_t)r);
    std::stable_sort(win.begin(), win.end(), [&](int32_t a, int32_t b) {
      return H.kt_ptr[a + 1] - H.kt_ptr[a] > H.kt_ptr[b + 1] - H.kt_ptr[b];
    });
    for (size_t a = 0; a < win.size(); a += SELL_H) {
      const size_t nr = std::min<size_t>(SELL_H, win.size() - a);
      int width = 0;
      for (size_t q = 0; q < nr; ++q) width = std::max(width, H.kt_ptr[win[a + q] + 1] - H.kt_ptr[win[a + q]]);
      width = (width + 3) / 4 * 4;
      const size_t base = col.size();
      if (base + (size_t)width * SELL_H >= (size_t)INT32_MAX) throw std::runtime_error("Poisson operator too large");
      col.resize(base + (size_t)width * SELL_H);
      val.resize(base + (size_t)width * SELL_H, 0.0);
      for (int q = 0; q < SELL_H; ++q) {
        const int32_t r = q < (int)nr ? win[a + q] : -1;
        row.push_back(r);
        const int beg = r >= 0 ? H.kt_ptr[r] : 0, len = r >= 0 ? H.kt_ptr[r + 1] - beg : 0;
        for (int t = 0; t < width; ++t) {
          const size_t e = base + (size_t)t * SELL_H + q;
          col[e] = t < len ? H.kt_col[beg + t] : std::max<int32_t>(r, 0);
          val[e] = t < len ? H.kt_val[beg + t] : 0.0;
        }
      }
      ptr.push_back((int32_t)col.size());
    }
  }
  d.sell_ptr = op->upload(ptr, s);
  d.sell_row = op->upload(row, s);
  d.sell_col = op->upload(col, s);
  d.sell_val = op->upload(val, s);
  const std::vector<float> valf(val.begin(), val.end());
  d.sell_valf = op->upload(valf, s);
  d.n_slices = (int64_t)ptr.size() - 1;
  HIPCHK(hipStreamSynchronize(s));  // the host tables are temporaries
}

extern "C" int mh_tune(mh_op* op, int32_t which, int32_t sched, int32_t grid_cap) {
  if (!op || which < 0 || which > 1 || sched < 0 || (sched & ~(which == 1 ? 1023 : 7)) != 0)
    return fail(MH_INVALID_ARG, "bad schedule");
  const int cap_max = 65536;
  if (grid_cap < 8 || grid_cap > cap_max) return fail(MH_INVALID_ARG, "grid_cap out of range");
  return guarded([&]() -> int {
    HIPCHK(hipDeviceSynchronize());
    if (which == 1 && (sched & 32) && !op->dh[0].sell_ptr) {
      for (int i = 0; i < op->ni; ++i) build_sell(op, i, nullptr);
      op->B.mx.n_slices = 0;
      for (const DevMesh& d : op->dh) op->B.mx.n_slices = std::max(op->B.mx.n_slices, d.n_slices);
    }
    for (DevMesh& d : op->dh) {
      if (which == 0) {
        d.sched_orb = sched;
        d.grid_orb = grid_cap;
      } else {
        d.sched_poi = sched;
        d.grid_poi = grid_cap;
      }
    }
    upload_instances(op, nullptr);
    return MH_OK;
  });
}

// ------------------------------------------------------------------ adjoint ----
// out = M^-1 Z u (dipole load vector through the mass solve), hanging rows filled
static void mass_dipole(mh_op* op, const double* u, double* out, hipStream_t s) {
  const Batch& B = op->B;
  stencil_orb(op, u, op->Ebuf, 3, 1, out, s);
  launch_ma_gather_orb(B, op->acc, 1, out, op->ma_b, s);
  launch_ma_solve(B, op->ma_b, op->ma_x, op->ma_r, op->ma_d0, op->ma_d1, nullptr, nullptr, out, s);
  launch_fill_orb(B, out, nullptr, s);
}

// out = M^-1 H1(E) u at the field value in Ebuf[0], hanging rows filled
static void mass_h1(mh_op* op, const double* u, double* out, hipStream_t s) {
  const Batch& B = op->B;
  stencil_orb(op, u, op->Ebuf, 1, 1, out, s);
  launch_ma_gather_orb(B, op->acc, 1, out, op->ma_b, s);
  launch_ma_solve(B, op->ma_b, op->ma_x, op->ma_r, op->ma_d0, op->ma_d1, nullptr, nullptr, out, s);
  launch_fill_orb(B, out, nullptr, s);
}

// out = M^-1 C^T f for a full-node load f given at the extended rows
static void mass_load(mh_op* op, const double* f, double* out, hipStream_t s) {
  const Batch& B = op->B;
  launch_load_split(B, f, out, op->acc, s);
  launch_ma_gather_orb(B, op->acc, 1, out, op->ma_b, s);
  launch_ma_solve(B, op->ma_b, op->ma_x, op->ma_r, op->ma_d0, op->ma_d1, nullptr, nullptr, out, s);
  launch_fill_orb(B, out, nullptr, s);
}

namespace {
struct DevScratch {
  std::vector<DevBlock> p;
  double* get(size_t nd) {
    p.push_back(dev_alloc(std::max<size_t>(nd, 2) * sizeof(double)));
    return (double*)p.back().p;
  }
  ~DevScratch() {
    (void)hipDeviceSynchronize();
    for (const DevBlock& b : p) dev_free(b);
  }
};
}  // namespace

// CG on the assembled Poisson operator for the right-hand side already in
// P.r (with the convergence targets in the SC_BB scalars), started from the
// DoF rows of the full-row array Z, which receive the solution.
static int cg_solve_rhs(mh_op* op, double* Z, int* iters, hipStream_t s) {
  const Batch& B = op->B;
  PoissonWs& P = op->P;
  launch_cg_start(B, Z, P.r, P, 1, s);
  const int conv = cg_iterate(op, Z, iters, s);
  if (conv < 0) return fail(MH_NONFINITE, "non-finite adjoint Poisson residual");
  return conv ? MH_OK : MH_NOT_CONVERGED;
}

extern "C" int mh_propagate_adjoint(mh_op* op, const double* phi0, const double* Ci0, double* W_work,
                                    const double* E_steps, int32_t n_steps, double dt, int32_t m,
                                    const double* dJ_dd, double* dJ_dE, int32_t n_quad, int32_t ckpt_stride,
                                    void* stream) {
  if (!op || !phi0 || !Ci0 || !W_work || !E_steps || !dJ_dd || !dJ_dE) return fail(MH_INVALID_ARG, "null argument");
  if (op->ni != 1) return fail(MH_UNSUPPORTED, "the adjoint takes a single instance");
  if (op->n > 4) return fail(MH_UNSUPPORTED, "the adjoint is implemented for at most 4 orbitals");
  if (op->ci.dim > 12) return fail(MH_UNSUPPORTED, "the adjoint needs an exact CI exponential (at most 12 determinants)");
  if (op->B.mx.gauge != MH_GAUGE_LENGTH) return fail(MH_UNSUPPORTED, "the adjoint is implemented in the length gauge");
  if (op->B.mx.ecs) return fail(MH_UNSUPPORTED, "the adjoint is implemented without complex scaling");
  if (n_steps < 1 || m < 1 || m > 24 || n_quad < 1 || n_quad > 16) return fail(MH_INVALID_ARG, "bad sizes");
  return guarded([&]() -> int {
    hipStream_t s = S(stream);
    const Batch& B = op->B;
    const int n = op->n, nn = n * n, ncol = op->ncol, dim = op->ci.dim;
    const int mci = std::min(12, dim);
    const size_t len = (size_t)2 * B.tE * n, clen = (size_t)2 * dim, wlen = (size_t)B.tF * ncol;
    const int S_ = ckpt_stride > 0 ? ckpt_stride : std::max(1, (int)std::lround(std::sqrt((double)n_steps)));
    int status = MH_OK;
    DevScratch mem;
    const int nck = n_steps / S_ + 1;
    std::vector<double*> ck(nck), ckC(nck), seg(S_ + 1), segC(S_ + 1), segW(S_);
    for (int i = 0; i < nck; ++i) { ck[i] = mem.get(len); ckC[i] = mem.get(clen); }
    for (int i = 0; i <= S_; ++i) { seg[i] = mem.get(len); segC[i] = mem.get(clen); }
    for (int i = 0; i < S_; ++i) segW[i] = mem.get(wlen);
    double* cur = mem.get(len), *curC = mem.get(clen);
    double* nu = mem.get(len), *va = mem.get(len), *vb = mem.get(len), *t1 = mem.get(len), *t2 = mem.get(len);
    double* Fc = mem.get(len), *Phib = mem.get(len);
    double* Q = mem.get((size_t)2 * B.tE * nn);
    double* Kw = mem.get(wlen), *Zb = mem.get(wlen);
    double* tb = mem.get((size_t)std::max<int64_t>(1, B.mx.Nb) * ncol);
    double* qlm = mem.get((size_t)op->P.nharm * ncol);
    double* qwpart = mem.get((size_t)qw_part_doubles(B));
    double* sm = mem.get((size_t)2 * ADJ_NBLK * nn);
    double* Kg = mem.get((size_t)2 * nn * nn), *KGam = mem.get((size_t)2 * nn * nn), *G2 = mem.get((size_t)2 * nn * nn);
    double* tgam = mem.get((size_t)2 * nn), *tGam = mem.get((size_t)2 * nn * nn);
    double* th = mem.get((size_t)2 * nn), *tg2 = mem.get((size_t)2 * nn * nn);
    double* Gz = mem.get((size_t)2 * nn), *Sm = mem.get((size_t)2 * nn);
    double* kap = mem.get(clen), *ca = mem.get(clen), *cb = mem.get(clen), *sig = mem.get(clen);
    double* DA = mem.get((size_t)2 * dim * nn), *DB = mem.get((size_t)2 * dim * nn);
    double* ebar = mem.get((size_t)n_steps + 1);
    launch_zero(ebar, n_steps + 1, s);
    launch_zero(Zb, wlen, s);
    double* XG = sm + 2 * ADJ_XG * nn, *XR = sm + 2 * ADJ_XR * nn, *L2 = sm + 2 * ADJ_LAM2 * nn;
    double* XL1 = sm + 2 * ADJ_XL1 * nn, *XL2 = sm + 2 * ADJ_XL2 * nn, *XH = sm + 2 * ADJ_XH * nn;
    double* XD = sm + 2 * ADJ_XD * nn, *KH = sm + 2 * ADJ_KH * nn;
    ensure_krylov(op, m);

    // one forward step of mh_propagate (real time), W warm-started from its contents
    auto fwd_step = [&](double* c, double* Cv, double* W, int k) -> int {
      launch_ci_rdm_full(1, op->ci, Cv, op->gam, op->Gam, op->Gtmp, s);
      int it = 0;
      const int rc = poisson_solve(op, c, W, 1, &it, s);
      if (rc < 0) return rc;
      if (rc == MH_NOT_CONVERGED) status = MH_NOT_CONVERGED;
      launch_set(op->Ebuf, E_steps[k], s);
      step_after_poisson(op, c, Cv, W, 1, dt, 0.0, m, 0, s);
      return MH_OK;
    };
    // x <- exp(+i tau G^H) x in the M inner product: G^H = R(gr^T) G'' R(ginv^T),
    // G'' = M^-1 H_F - R(lam2) (the forward operator with the mixing lam2)
    auto adj_exp = [&](double* x, double tau) {
      launch_mix(B, x, XG, 0.0, t2, s);
      double* lam_alt = L2;
      std::swap(op->lam, lam_alt);
      arnoldi(op, t2, -tau, 0.0, m, s);
      std::swap(op->lam, lam_alt);
      launch_mix(B, t2, XR, 0.0, x, s);
    };

    // forward sweep with checkpoints every S_ steps
    launch_copy(phi0, cur, len, s);
    launch_copy(Ci0, curC, clen, s);
    for (int k = 0; k < n_steps; ++k) {
      if (k % S_ == 0) {
        launch_copy(cur, ck[k / S_], len, s);
        launch_copy(curC, ckC[k / S_], clen, s);
      }
      const int rc = fwd_step(cur, curC, W_work, k);
      if (rc < 0) return rc;
    }
    // terminal adjoint state from d_N
    launch_ci_rdm_full(1, op->ci, curC, op->gam, op->Gam, op->Gtmp, s);
    launch_gram(B, cur, cur, WT_DIPOLE, ROWS_EXT, op->gpart, gram_blocks(B.mx.NE), op->zmat, s);
    launch_zero(sm, 2 * ADJ_NBLK * nn, s);
    launch_zero(KGam, 2 * nn * nn, s);
    launch_adj_terms(op->zmat, op->gam, dJ_dd[n_steps], n, ebar + n_steps, sm, s);
    launch_mix(B, cur, XD, 0.0, t1, s);
    mass_dipole(op, t1, nu, s);
    launch_adj_ciprep(sm, KGam, n, th, tg2, s);
    launch_ci_apply(1, op->ci, th, tg2, curC, kap, s);

    std::vector<double> gx, gw;
    gauss_legendre(n_quad, gx, gw);
    for (int j = 0; j < n_quad; ++j) {
      gx[j] = 0.5 * (gx[j] + 1.0);
      gw[j] *= 0.5;
    }
    for (int s0 = ((n_steps - 1) / S_) * S_; s0 >= 0; s0 -= S_) {
      const int s1 = std::min(s0 + S_, n_steps);
      // recompute the segment: states and pair potentials of steps s0 .. s1-1
      launch_copy(ck[s0 / S_], seg[0], len, s);
      launch_copy(ckC[s0 / S_], segC[0], clen, s);
      for (int k = s0; k < s1; ++k) {
        const int j = k - s0;
        launch_copy(j == 0 ? W_work : segW[j - 1], segW[j], wlen, s);
        launch_ci_rdm_full(1, op->ci, segC[j], op->gam, op->Gam, op->Gtmp, s);
        int it = 0;
        const int rc = poisson_solve(op, seg[j], segW[j], 1, &it, s);
        if (rc < 0) return rc;
        if (rc == MH_NOT_CONVERGED) status = MH_NOT_CONVERGED;
        if (k + 1 < s1) {
          launch_copy(seg[j], seg[j + 1], len, s);
          launch_copy(segC[j], segC[j + 1], clen, s);
          launch_set(op->Ebuf, E_steps[k], s);
          step_after_poisson(op, seg[j + 1], segC[j + 1], segW[j], 1, dt, 0.0, m, 0, s);
        }
      }
      for (int k = s1 - 1; k >= s0; --k) {
        double* c = seg[k - s0];
        double* Cv = segC[k - s0];
        double* W = segW[k - s0];
        const double g = dJ_dd[k];
        launch_zero(sm, 2 * ADJ_NBLK * nn, s);
        launch_zero(Kg, 2 * nn * nn, s);
        launch_zero(Q, 2 * B.tE * nn, s);
        // frozen data, integrals and observables of step k
        launch_ci_rdm_full(1, op->ci, Cv, op->gam, op->Gam, op->Gtmp, s);
        launch_set(op->Ebuf, E_steps[k], s);
        freeze_body(op, c, op->gam, op->Gam, W, s);
        load_vector(op, c, op->Ebuf, 1, op->F, s);
        launch_gram(B, c, op->F, WT_NONE, ROWS_DOF, op->gpart, gram_blocks(B.mx.N), op->hmat, s);
        launch_gint_full(B, c, W, op->colmap, op->gpart, gint_blocks(B), op->Gtmp, op->gint, s);
        launch_gram(B, c, c, WT_DIPOLE, ROWS_EXT, op->gpart, gram_blocks(B.mx.NE), op->zmat, s);
        launch_ci_hprime(1, op->ci, op->hmat, op->gint, s);
        g_apply(op, c, Fc, 0, s);
        launch_adj_prep(op->ginv, op->lam, n, sm, s);
        // orbital exponential: Frechet quadrature, then nu_k = exp(+i dt G^H) nu_{k+1}
        for (int j = 0; j < n_quad; ++j) {
          const double wi = -dt * gw[j];  // omega_j = -i dt w_j
          launch_copy(c, vb, len, s);
          arnoldi(op, vb, gx[j] * dt, 0.0, m, s);
          launch_copy(nu, va, len, s);
          adj_exp(va, (1.0 - gx[j]) * dt);
          launch_gram(B, va, vb, WT_DIPOLE, ROWS_EXT, op->gpart, gram_blocks(B.mx.NE), Gz, s);
          launch_gram(B, va, vb, WT_MASS, ROWS_EXT, op->gpart, gram_blocks(B.mx.NE), Sm, s);
          launch_adj_quad(Gz, Sm, 0.0, wi, n, ebar + k, sm, s);
          launch_q_accum(B, va, vb, 0.0, wi, Q, s);
        }
        adj_exp(nu, dt);
        // CI exponential: the same quadrature, then kappa_k = exp(+i dt H) kappa_{k+1}
        for (int j = 0; j < n_quad; ++j) {
          const double wi = -dt * gw[j];
          launch_copy(kap, ca, clen, s);
          launch_ci_lanczos(1, op->ci, op->Qdev, op->Qh.data(), mci, op->gint, ca, op->KC, -(1.0 - gx[j]) * dt, 0.0,
                            0, s);
          launch_copy(Cv, cb, clen, s);
          launch_ci_lanczos(1, op->ci, op->Qdev, op->Qh.data(), mci, op->gint, cb, op->KC, gx[j] * dt, 0.0, 0, s);
          launch_ci_trdm(1, op->ci, ca, cb, DA, DB, tgam, tGam, op->Gtmp, s);
          launch_caxpy(nn, 0.0, wi, tgam, KH, s);
          launch_caxpy((int64_t)nn * nn, 0.0, 0.5 * wi, tGam, Kg, s);
        }
        launch_ci_lanczos(1, op->ci, op->Qdev, op->Qh.data(), mci, op->gint, kap, op->KC, -dt, 0.0, 0, s);
        // lambda, h and dipole terms
        launch_adj_terms(op->zmat, op->gam, g, n, ebar + k, sm, s);
        launch_mix(B, Fc, XL1, 1.0, nu, s);             // nu += (M^-1 F(c)) Lbar^T
        launch_mix(B, c, XL2, 0.0, t1, s);              // Y = c conj(Lbar)
        launch_q_accum(B, t1, c, 1.0, 0.0, Q, s);
        launch_mix(B, t1, XG, 0.0, t2, s);
        g_apply(op, t2, va, 0, s);
        launch_mix(B, va, XR, 1.0, nu, s);              // nu += M^-1 H_F^H Y
        launch_mix(B, c, XH, 0.0, t1, s);
        mass_h1(op, t1, va, s);
        launch_axpby(len, 1.0, va, 1.0, nu, s);
        launch_mix(B, c, XD, 0.0, t1, s);
        mass_dipole(op, t1, va, s);
        launch_axpby(len, 1.0, va, 1.0, nu, s);
        // mean field: sensitivities of the pair potentials, gamma^-1 and Gamma
        launch_zero(Kw, wlen, s);
        launch_adj_mf(B, Q, W, c, op->ginv, op->Mr, Kg, op->colmap, Kw, Phib, s);
        launch_qw_gram(B, Q, W, qwpart, G2, s);
        launch_adj_mf_small(G2, op->Mr, op->ginv, op->colmap, n, sm, KGam, s);
        // pair Poisson solves, reversed
        launch_adj_poisson_rhs(B, Kw, ncol, op->P.r, op->P.sc, s);
        int it = 0;  // started from the previous step's solution (zero at the first)
        const int rc = cg_solve_rhs(op, Zb, &it, s);
        if (rc < 0) return rc;
        if (rc == MH_NOT_CONVERGED) status = MH_NOT_CONVERGED;
        launch_fill_real(B, Zb, 1, ncol, 1, nullptr, s);
        launch_zero(tb, (int64_t)std::max<int64_t>(1, B.mx.Nb) * ncol, s);
        launch_adj_bnd(B, Kw, Zb, ncol, op->P.nharm, tb, qlm, s);
        launch_krho(B, Zb, qlm, op->P.lmax, ncol, op->colmap, c, Phib, s);
        mass_load(op, Phib, va, s);
        launch_axpby(len, 1.0, va, 1.0, nu, s);
        // CI: the RDM sensitivities as an operator on C_k
        launch_adj_ciprep(sm, KGam, n, th, tg2, s);
        launch_ci_apply(1, op->ci, th, tg2, Cv, sig, s);
        launch_axpby(clen, 1.0, sig, 1.0, kap, s);
      }
    }
    std::vector<double> eb((size_t)n_steps + 1);
    HIPCHK(hipMemcpyAsync(eb.data(), ebar, eb.size() * sizeof(double), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    const double E0 = op->dh[0].E0;
    for (int k = 0; k < n_steps; ++k) dJ_dE[k] = E0 * eb[k];
    return status;
  });
}
