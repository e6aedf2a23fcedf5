// lbm.hip -- host side of the C ABI declared in include/lbm.h.
//
// A context owns (or borrows) one device workspace that holds everything the
// step keeps resident: the two population arrays (AA, structure-of-arrays),
// phi, the repulsive flux J, the near-contact tile flags and lists, and the
// reduction scratch.  Each step enqueues k_phi, k_nci (when A_rep != 0) and
// k_collide on the context's stream; every diag_interval steps the collide
// kernel also produces FP64 partial sums and k_diag / k_reduce finish them.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <type_traits>
#include <vector>

#include "../../include/lbm.h"
#include "kernels.hpp"
#include "stats.hpp"

using namespace lbm;

namespace {

constexpr int HIST = 64;      // periodic diagnostics kept on the device
constexpr int NCI_GRID = 4096;   // near-contact blocks (512^3 swarm: 0.291 ms against 0.314 with 2048)
// Near-contact tiles from which a lattice selects them before the near-contact
// pass (below, the two extra launches cost more than the pass saves: the steps of
// 64^3 to 192^3 lattices are bound by launch latency).
constexpr int NCI_SELECT_TILES = 16384;
constexpr int RED1 = 512;     // first-stage blocks of the diagnostic reduction

thread_local std::string g_create_error;

size_t align256(size_t v) { return (v + 255) & ~size_t(255); }

int q_hydro(int dim) { return dim == 2 ? 9 : 19; }
int q_hydro(const lbm_params* p) { return p->dim == 2 ? 9 : (p->hydro_q == 27 ? 27 : 19); }
int q_phase(int dim) { return dim == 2 ? 9 : 7; }

size_t real_size(int prec) { return prec == LBM_FP64 ? 8 : 4; }
size_t fstore_size(int prec) { return prec == LBM_FP64 ? 8 : (prec == LBM_FP32 ? 4 : 2); }

// Near-contact tile of a lattice: the kernels' NciTile of its dimension and
// arithmetic type (FP64, or FP32 for every other precision).
template <int DIM, typename T>
void tile_dims_of(int* tx, int* ty, int* tz) {
  *tx = NciTile<DIM, T>::TX;
  *ty = NciTile<DIM, T>::TY;
  *tz = NciTile<DIM, T>::TZ;
}
void tile_dims(int dim, int prec, int* tx, int* ty, int* tz) {
  if (dim == 2)
    prec == LBM_FP64 ? tile_dims_of<2, double>(tx, ty, tz) : tile_dims_of<2, float>(tx, ty, tz);
  else
    prec == LBM_FP64 ? tile_dims_of<3, double>(tx, ty, tz) : tile_dims_of<3, float>(tx, ty, tz);
}

struct Layout {
  long long N, S;
  int nblk, ntiles, ttx, tty, ttz, ntx, nty, ntz;
  int rs, qc;   // population chunks: 2^rs rows, qc = nx 2^rs cells
  int bxs;      // cell-wise blocks are 2^bxs cells wide
  size_t off_f, off_g, off_phi, off_J, off_flags, off_list, off_cnt, off_pa, off_pb, off_s1,
      off_red, off_lab, off_phi2, off_ua, off_srng, off_alist, total;
};

bool valid_params(const lbm_params* p, std::string* why) {
  auto bad = [&](const char* m) {
    if (why) *why = m;
    return false;
  };
  if (!p) return bad("null parameters");
  if (p->dim != 2 && p->dim != 3) return bad("dim must be 2 or 3");
  if (p->nx < 1 || p->ny < 1 || p->nz < 1) return bad("box sizes must be positive");
  if (p->dim == 2 && p->nz != 1) return bad("2D boxes need nz = 1");
  const long long N = (long long)p->nx * p->ny * p->nz;
  if (N >= (1LL << 31) - 4096) return bad("box too large (more than 2^31 cells)");
  if (p->dim == 3 ? (p->hydro_q != 0 && p->hydro_q != 19 && p->hydro_q != 27)
                  : (p->hydro_q != 0 && p->hydro_q != 9))
    return bad("hydro_q must be 0, 19 or 27 in 3D (0 or 9 in 2D)");
  if ((long long)p->nx * p->ny * q_hydro(p) >= (1LL << 32))
    return bad("z plane too large (nx ny q must be below 2^32)");
  if (p->precision < LBM_FP64 || p->precision > LBM_FP32_BF16STORE) return bad("unknown precision");
  if (!(p->tau > 0.5)) return bad("tau must exceed 1/2");
  if (!(p->visc_ratio > 0)) return bad("visc_ratio must be positive");
  if (!(p->mobility > 0)) return bad("mobility must be positive");
  if (!(p->width > 0)) return bad("width must be positive");
  if (!(p->sigma >= 0)) return bad("sigma must be non-negative");
  if (!(p->density_ratio > 0)) return bad("density_ratio must be positive");
  if (!(p->a_rep >= 0)) return bad("a_rep must be non-negative");
  if (p->nci_window < 1 || p->nci_window > 3) return bad("nci_window must be 1, 2 or 3");
  if (!(p->h0 > 0) || !(p->p_exp > 0)) return bad("h0 and p_exp must be positive");
  if (!(p->eps_q >= 0) || !(p->eps_q < 0.125) || !(p->eps_n >= 0)) return bad("bad eps_q / eps_n");
  if (!(p->tie_eps >= 0) || !(p->tie_eps < 0.1)) return bad("tie_eps must be in [0, 0.1)");
  if (p->rep_orient < -1 || p->rep_orient > 1) return bad("rep_orient must be -1, 0 or 1");
  if (p->dispersed < -1 || p->dispersed > 1) return bad("dispersed must be -1, 0 or 1");
  if (p->diag_interval < 0) return bad("diag_interval must be >= 0");
  if (p->cac_solver != 0 && p->cac_solver != 1) return bad("cac_solver must be 0 or 1");
  if (p->hydro_store != 0 && p->hydro_store != 1) return bad("hydro_store must be 0 or 1");
  return true;
}

// Combinations that are valid but not built: moment storage runs in 3D, with
// FP64 or FP32 coefficients and the lattice Boltzmann phase field.
bool supported(const lbm_params* p, std::string* why) {
  if (p->hydro_store == 1 && (p->dim != 3 || (p->precision != LBM_FP64 && p->precision != LBM_FP32) ||
                              p->cac_solver != 0)) {
    *why = "moment storage (hydro_store 1) needs dim 3, FP64 or FP32, and cac_solver 0";
    return false;
  }
  return true;
}

// Width of the cell-wise blocks: the widest of 256, 128, 64 cells that leaves
// at most 1/8 of the lanes of a row idle (256 at nx = 512; 64 for narrow boxes).
int block_shift(int nx) {
  for (int s = 8; s > 6; --s) {
    const int w = 1 << s;
    if ((long long)((nx + w - 1) / w) * w * 8 <= (long long)nx * 9) return s;
  }
  return 6;
}

Layout make_layout(const lbm_params* p) {
  Layout L{};
  L.N = (long long)p->nx * p->ny * p->nz;
  // Plane stride: N rounded up to 128 plus 1088 elements (a 256-byte multiple in
  // FP32), so that the 26 concurrent population streams do not start at the same
  // offset modulo large powers of two (+4 % on the collide kernel at 512^3).
  L.S = ((L.N + 127) & ~127LL) + 1088;
  // Population chunks of about 8192 cells (2^rs rows; rs no larger than the
  // power of two dividing ny, so no chunk is partial): a block's 26 population
  // streams then fall into a few contiguous regions (+8 % streaming bandwidth
  // over planes of the whole box, measured at 512^3).
  {
    int lg = 0;
    while ((1 << lg) < p->nx) ++lg;
    int tz = 0;
    while (tz < 30 && ((p->ny >> tz) & 1) == 0) ++tz;
    L.rs = std::min(std::max(0, 13 - lg), tz);
    L.qc = p->nx << L.rs;
  }
  L.bxs = block_shift(p->nx);
  const int bw = 1 << L.bxs, bh = NT >> L.bxs;
  const int nbx = (p->nx + bw - 1) / bw, nby = (p->ny + bh - 1) / bh;
  L.nblk = nbx * nby * p->nz;
  tile_dims(p->dim, p->precision, &L.ttx, &L.tty, &L.ttz);
  L.ntx = (p->nx + L.ttx - 1) / L.ttx;
  L.nty = (p->ny + L.tty - 1) / L.tty;
  L.ntz = (p->nz + L.ttz - 1) / L.ttz;
  L.ntiles = L.ntx * L.nty * L.ntz;
  const size_t rs = real_size(p->precision), fs = fstore_size(p->precision);
  size_t o = 0;
  // populations f (AA, one copy), or with moment storage two buffers of NMOM
  // coefficient planes
  L.off_f = o;
  o = align256(o + (p->hydro_store ? 2 * (size_t)NMOM * L.S * rs : (size_t)q_hydro(p) * L.N * fs));
  L.off_g = o;   o = align256(o + (size_t)q_phase(p->dim) * L.N * rs);
  L.off_phi = o; o = align256(o + (size_t)L.S * rs);
  L.off_J = o;   o = align256(o + (size_t)p->dim * L.S * rs);
  L.off_flags = o; o = align256(o + 2 * (size_t)L.ntiles * 4);
  L.off_list = o;  o = align256(o + 2 * (size_t)L.ntiles * 4);
  L.off_cnt = o;   o = align256(o + 64);
  L.off_pa = o;    o = align256(o + (size_t)L.nblk * NPART * 8);
  L.off_pb = o;    o = align256(o + (size_t)L.nblk * NPART * 8);
  L.off_s1 = o;    o = align256(o + 2 * (size_t)RED1 * NPART * 8);
  L.off_red = o;   o = align256(o + (size_t)(HIST + 1) * 2 * NPART * 8);
  L.off_lab = o;   o = align256(o + (size_t)L.N * 4);
  // finite-difference phase field only: the second phi buffer and the u planes
  const bool fd = p->cac_solver != 0;
  L.off_phi2 = o;  o = align256(o + (fd ? (size_t)L.S * rs : 0));
  L.off_ua = o;    o = align256(o + (fd ? (size_t)p->dim * L.S * rs : 0));
  // near-contact tile selection: normal ranges per sub-tile, the selected tiles
  L.off_srng = o;  o = align256(o + (size_t)L.ntiles * (p->dim == 3 ? 8 : 4) * 6 * rs);
  L.off_alist = o; o = align256(o + (size_t)L.ntiles * 4);
  L.total = o;
  return L;
}

}  // namespace

struct lbm_ctx {
  lbm_params p;
  Layout L;
  int dev = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  char* ws = nullptr;
  bool own_ws = false;
  Geo geo{};
  Phys phys{};
  NciP nci{};
  long step = 0;
  bool initialised = false;
  int dispersed = 1;
  long hist_step[HIST];
  int hist_count = 0;   // diagnostics recorded since the last reset
  std::string err;
  // per-kernel event timing
  bool timing = false;
  std::vector<hipEvent_t> ev;      // pairs (start, stop)
  std::vector<int> ev_kind;
  int ev_used = 0;
  double k_ms[5] = {0, 0, 0, 0, 0};
  long k_cnt[5] = {0, 0, 0, 0, 0};
  int phi_cur = 0;   // finite-difference phase field: which phi buffer holds the state
  bool wide_offsets = false;   // lbm_force_wide_offsets: 64-bit offset kernels at any size
  int nci_select = -1;         // lbm_nci_select: -1 by size, 0 never, 1 always
  int mom_cur = 0;   // moment storage: which coefficient buffer holds the state

  void* f() const { return ws + L.off_f; }
  void* g() const { return ws + L.off_g; }
  void* phi() const { return ws + (phi_cur ? L.off_phi2 : L.off_phi); }
  void* phi_next() const { return ws + (phi_cur ? L.off_phi : L.off_phi2); }
  void* ua() const { return ws + L.off_ua; }
  bool fd() const { return p.cac_solver != 0; }
  bool mom() const { return p.hydro_store != 0; }
  // coefficient buffer k of the moment storage (NMOM planes of stride S)
  void* mom_buf(int k) const { return ws + L.off_f + (size_t)k * NMOM * L.S * real_size(p.precision); }
  void* J() const { return ws + L.off_J; }
  unsigned* flags(int k) const { return (unsigned*)(ws + L.off_flags) + (size_t)k * L.ntiles; }
  unsigned* list(int k) const { return (unsigned*)(ws + L.off_list) + (size_t)k * L.ntiles; }
  // [0], [1] tile lists per parity, [2] cells with a partner, [3] tiles selected for
  // the near-contact pass, [6] tiles the previous near-contact pass took
  unsigned* cnt() const { return (unsigned*)(ws + L.off_cnt); }
  void* srng() const { return ws + L.off_srng; }
  unsigned* alist() const { return (unsigned*)(ws + L.off_alist); }
  double* pa() const { return (double*)(ws + L.off_pa); }
  double* pb() const { return (double*)(ws + L.off_pb); }
  double* s1(int k) const { return (double*)(ws + L.off_s1) + (size_t)k * RED1 * NPART; }
  double* red(int slot) const { return (double*)(ws + L.off_red) + (size_t)slot * 2 * NPART; }
  unsigned* lab() const { return (unsigned*)(ws + L.off_lab); }   // component labels (diagnostics)
  bool nci_on() const { return p.a_rep > 0.0; }
  int fail(int code, const std::string& m) {
    err = m;
    return code;
  }
};

#define HIP_OR_FAIL(ctx, expr)                                                             \
  do {                                                                                     \
    hipError_t e_ = (expr);                                                                \
    if (e_ != hipSuccess) return (ctx)->fail(LBM_E_HIP, std::string(#expr ": ") + hipGetErrorString(e_)); \
  } while (0)

namespace {

constexpr int EV_PAIRS = 2048;

int flush_timing(lbm_ctx* c) {
  if (c->ev_used == 0) return LBM_OK;
  HIP_OR_FAIL(c, hipStreamSynchronize(c->stream));
  for (int k = 0; k < c->ev_used; ++k) {
    float ms = 0.f;
    HIP_OR_FAIL(c, hipEventElapsedTime(&ms, c->ev[2 * k], c->ev[2 * k + 1]));
    c->k_ms[c->ev_kind[k]] += ms;
    c->k_cnt[c->ev_kind[k]] += 1;
  }
  c->ev_used = 0;
  return LBM_OK;
}

// Brackets one launch with a pair of events when timing is on.
struct Timed {
  lbm_ctx* c;
  int slot = -1;
  Timed(lbm_ctx* c_, int kind) : c(c_) {
    if (!c->timing) return;
    if (c->ev_used == EV_PAIRS) flush_timing(c);
    slot = c->ev_used++;
    c->ev_kind[slot] = kind;
    (void)hipEventRecord(c->ev[2 * slot], c->stream);
  }
  ~Timed() {
    if (slot >= 0) (void)hipEventRecord(c->ev[2 * slot + 1], c->stream);
  }
};

// ---------------------------------------------------------------------------
// Batches of lattices stepped together (serving)
// ---------------------------------------------------------------------------

constexpr int BATCH_R = 8;        // steps per captured graph replay
constexpr int BATCH_CACHE = 8;    // cached batches (job tables and graphs)

// Device job table, its pinned host mirror and the captured replay graph of one
// ordered set of contexts.  A graph bakes the table pointer and the grid sizes;
// the table contents (step counters) are re-uploaded before every call.
struct Batch {
  std::vector<lbm_ctx*> ctxs;
  void* djobs = nullptr;
  void* hjobs = nullptr;
  size_t bytes = 0;
  int total_blocks = -1;
  bool o32 = false;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  hipEvent_t done = nullptr;     // end of the last call's work
  hipEvent_t copied = nullptr;   // the last call's upload of the job table has run
  bool used = false;
  ~Batch() {
    if (used && done) (void)hipEventSynchronize(done);   // no launch may still read the table
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    if (djobs) (void)hipFree(djobs);
    if (hjobs) (void)hipHostFree(hjobs);
    if (done) (void)hipEventDestroy(done);
    if (copied) (void)hipEventDestroy(copied);
  }
};

std::vector<Batch*>& batches() {
  static std::vector<Batch*> b;
  return b;
}

void forget_batches_of(const lbm_ctx* c) {
  auto& bs = batches();
  for (size_t i = 0; i < bs.size();) {
    bool has = false;
    for (lbm_ctx* x : bs[i]->ctxs) has |= (x == c);
    if (has) {
      delete bs[i];
      bs.erase(bs.begin() + (long)i);
    } else {
      ++i;
    }
  }
}

// ---------------------------------------------------------------------------
// The job table of lbm_batch_step_noalloc: a fixed device array instead of an
// allocation.  Host code never passes the array's name to a kernel or a copy:
// it takes the array's address on each device once, with hipGetSymbolAddress,
// and uses that pointer.
// ---------------------------------------------------------------------------

constexpr int STATIC_JOBS = 64;               // most contexts one call may advance
constexpr size_t STATIC_JOB_BYTES = 1024;     // room per table entry (any precision)
static __device__ __align__(256) unsigned char scratch[STATIC_JOBS * STATIC_JOB_BYTES];

constexpr int MAX_DEVICES = 64;
void* g_scratch_ptr[MAX_DEVICES] = {};

// Address of this device's copy of the table, taken once per device with that
// device current (the caller's current device is restored).
int scratch_on(int dev, void** out, std::string* why) {
  if (dev < 0 || dev >= MAX_DEVICES) {
    *why = "device ordinal beyond the static table's device list";
    return LBM_E_UNSUPPORTED;
  }
  if (!g_scratch_ptr[dev]) {
    int cur = 0;
    if (hipGetDevice(&cur) != hipSuccess || (cur != dev && hipSetDevice(dev) != hipSuccess)) {
      *why = "cannot make the context's device current";
      return LBM_E_HIP;
    }
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (cur != dev) (void)hipSetDevice(cur);
    if (e != hipSuccess || !ptr) {
      *why = std::string("hipGetSymbolAddress of the static job table: ") + hipGetErrorString(e);
      return LBM_E_HIP;
    }
    g_scratch_ptr[dev] = ptr;
  }
  *out = g_scratch_ptr[dev];
  return LBM_OK;
}

// Table entries passed by value: K of them per launch, so that the kernel
// arguments stay within 2 KB.
template <typename JT, int K>
struct JobChunk {
  JT j[K];
};
template <typename JT, int K>
__global__ void k_put_jobs(JT* __restrict__ dst, JobChunk<JT, K> c, int n) {
  const int t = threadIdx.x;
  if (t < n) dst[t] = c.j[t];
}

// ---------------------------------------------------------------------------
// Typed launch sequences
// ---------------------------------------------------------------------------

template <typename T>
int copy_field_to_host(lbm_ctx* c, const T* dsrc, long long comps, double* out) {
  const long long N = c->L.N, S = c->L.S;
  std::vector<T> h((size_t)comps * S);
  HIP_OR_FAIL(c, hipMemcpyAsync(h.data(), dsrc, sizeof(T) * comps * S, hipMemcpyDeviceToHost, c->stream));
  HIP_OR_FAIL(c, hipStreamSynchronize(c->stream));
  for (long long a = 0; a < comps; ++a)
    for (long long i = 0; i < N; ++i) out[a * N + i] = (double)h[(size_t)(a * S + i)];
  return LBM_OK;
}

void fill_diag(const double* r, long step, lbm_diag* d) {
  std::memset(d, 0, sizeof(*d));
  d->step = step;
  d->sum_pstar = r[0];
  d->momentum[0] = r[1];
  d->momentum[1] = r[2];
  d->momentum[2] = r[3];
  d->kinetic_energy = r[4];
  d->max_speed = r[5];
  d->nci_active = (long)r[7];
  d->mass_phi = r[NPART + 0];
  d->n_droplets = (long)std::llround(r[NPART + 1]);
  d->finite = (r[6] == 0.0 && r[NPART + 6] == 0.0 && std::isfinite(r[NPART + 0])) ? 1 : 0;
  d->film_cells = r[8];
  d->film_frep_n = r[9];
  d->film_fcap_n = r[10];
  d->film_frep = r[11];
  d->max_frep = r[12];
}

template <int DIM, int QH, typename T, typename FS, typename GS>
struct Engine {
  static dim3 rows(const lbm_ctx* c) { return dim3((unsigned)c->L.nblk); }

  // The mixture and forcing constants in the kernel's arithmetic type.
  static PhysT<T> physT(const lbm_ctx* c) {
    const Phys& P = c->phys;
    PhysT<T> q{};
    q.rho_g = (T)P.rho_g;
    q.drho = (T)P.drho;
    q.mu_a = (T)P.mu_a;
    q.mu_b = (T)P.mu_b;
    q.beta4 = (T)P.beta4;
    q.kappa = (T)P.kappa;
    q.rho_mean = (T)P.rho_mean;
    for (int a = 0; a < 3; ++a) q.g[a] = (T)P.g[a];
    q.kc = (T)P.kc;
    q.inv_tau_phi = (T)P.inv_tau_phi;
    q.eps_n = (T)P.eps_n;
    for (int i = 0; i < HydroQ<QH>::Q; ++i) q.fref[i] = (T)(HydroQ<QH>::w[i] * P.pstar_ref);
    return q;
  }

  // phi of the current state, plus (when the near-contact force is on) the
  // interfacial tile list of this parity.
  static void phi_pass(lbm_ctx* c, int par) {
    const int nci = c->nci_on() ? 1 : 0;
    // with the finite-difference phase field phi is the state: flags only
    auto k = c->fd() ? k_phi<DIM, 0, T, GS, true>
                     : (par == 0 ? k_phi<DIM, 0, T, GS, false> : k_phi<DIM, 1, T, GS, false>);
    Timed tm(c, 0);
    hipLaunchKernelGGL(k, rows(c), dim3(NT), 0, c->stream, (const GS*)c->g(), (T*)c->phi(), c->geo,
                       c->flags(par), c->list(par), c->cnt() + par, c->cnt() + 2, nci,
                       (T)c->p.q_th);
  }

  // Whether the near-contact pass selects tiles: on lattices of at least
  // NCI_SELECT_TILES tiles (lbm_nci_select can force it on or off).
  static bool nci_selects(const lbm_ctx* c) {
    return c->nci_select >= 0 ? c->nci_select != 0 : c->L.ntiles >= NCI_SELECT_TILES;
  }

  // Near-contact pass: normal ranges of the listed tiles, the tiles that can
  // hold a partner (the others flagged NCI_SKIPPED), then k_nci on those.
  static void nci_pass(lbm_ctx* c, int par, int* chi, int* part) {
    if (!c->nci_on()) return;
    const int grid = std::min(NCI_GRID, std::max(1, c->L.ntiles));
    Timed tm(c, 1);
    if (!nci_selects(c)) {
      // every listed tile (a small lattice's steps are bound by launches, not by this pass)
      if (chi)
        hipLaunchKernelGGL((k_nci<DIM, QH, T, true>), dim3(grid), dim3(NT_NCI), 0, c->stream,
                           (const T*)c->phi(), (T*)c->J(), chi, part, c->list(par), c->cnt() + par,
                           c->flags(1 - par), c->list(1 - par), c->cnt() + (1 - par), c->cnt() + 2,
                           c->geo, c->nci);
      else
        hipLaunchKernelGGL((k_nci<DIM, QH, T, false>), dim3(grid), dim3(NT_NCI), 0, c->stream,
                           (const T*)c->phi(), (T*)c->J(), (int*)nullptr, (int*)nullptr, c->list(par),
                           c->cnt() + par, c->flags(1 - par), c->list(1 - par), c->cnt() + (1 - par),
                           c->cnt() + 2, c->geo, c->nci);
      return;
    }
    // selection statistics of the previous pass: its list count (reset by the
    // collide after this pass) and the tiles it took (kept by the phi pass)
    const unsigned* prev_listed = c->cnt() + (1 - par);
    const unsigned* prev_taken = c->cnt() + 6;
    const int probe = (c->step & 31) == 0 ? 1 : 0;
    hipLaunchKernelGGL((k_nci_ranges<DIM, QH, T>), dim3(grid), dim3(NT_NCI), 0, c->stream, (const T*)c->phi(),
                       c->geo, (const unsigned*)c->list(par), (const unsigned*)(c->cnt() + par), (T*)c->srng(),
                       (T)c->p.q_th, (T)c->p.eps_n, prev_listed, prev_taken, probe);
    const int sgrid = std::min(NCI_GRID, std::max(1, (c->L.ntiles + 3) / 4));   // four waves per block
    hipLaunchKernelGGL((k_nci_select<DIM, T>), dim3(sgrid), dim3(256), 0, c->stream, c->geo, c->flags(par),
                       (const unsigned*)c->list(par), (const unsigned*)(c->cnt() + par), (const T*)c->srng(),
                       c->alist(), c->cnt() + 3, c->p.nci_window, (T)c->p.cos_opp, prev_listed, prev_taken, probe);
    if (chi) {
      hipLaunchKernelGGL((k_nci<DIM, QH, T, true>), dim3(grid), dim3(NT_NCI), 0, c->stream,
                         (const T*)c->phi(), (T*)c->J(), chi, part, c->alist(), c->cnt() + 3,
                         c->flags(1 - par), c->list(1 - par), c->cnt() + (1 - par), c->cnt() + 2,
                         c->geo, c->nci);
    } else {
      hipLaunchKernelGGL((k_nci<DIM, QH, T, false>), dim3(grid), dim3(NT_NCI), 0, c->stream,
                         (const T*)c->phi(), (T*)c->J(), (int*)nullptr, (int*)nullptr, c->alist(),
                         c->cnt() + 3, c->flags(1 - par), c->list(1 - par), c->cnt() + (1 - par),
                         c->cnt() + 2, c->geo, c->nci);
    }
  }

  static Planes<FS, GS> planes(const lbm_ctx* c) {
    Planes<FS, GS> pl{};
    pl.f = (FS*)c->f();
    pl.g = (GS*)c->g();
    return pl;
  }

  // 32-bit byte offsets are used when the populations of a z plane and every
  // phi / J plane stay below 4 GiB (and lbm_force_wide_offsets has not asked
  // for the 64-bit kernels).
  static bool off32(const lbm_ctx* c) {
    if (c->wide_offsets) return false;
    const size_t plane = (size_t)c->p.nx * c->p.ny;
    const size_t widest = std::max(plane * HydroQ<QH>::Q * sizeof(FS),
                                   std::max(plane * Phase<DIM>::Q * sizeof(GS), (size_t)c->L.S * sizeof(T)));
    return widest < (size_t(1) << 32);
  }

  // The odd parity's plain step runs one block per x row (k_collide_row) when
  // the staged rows fit in 64 KB of LDS and a row fills a block.  D3Q19 with
  // 4-byte populations in rows of a multiple of 512 cells uses 512-thread blocks
  // (at 512^3 FP32 the step ran 0.5 % faster); every other case 256 (with 16-bit
  // populations and with D3Q27, 512 threads were slower).
  static bool row_collide(const lbm_ctx* c) {
    if constexpr (DIM != 3) return false;
    const int nx = c->p.nx;
    return nx >= NT && nx % 64 == 0 && xrow_bytes<DIM, QH, FS, GS>(nx) <= 64u * 1024u;
  }

  template <int MODE>
  static void collide_pass(lbm_ctx* c, int par, T* macro) {
    if constexpr (DIM == 3 && std::is_same<FS, T>::value && std::is_same<GS, T>::value) {
      if (c->mom()) {
        const bool o32 = off32(c);
        auto k = par == 0 ? (o32 ? k_collide_mom<QH, 0, MODE, T, true> : k_collide_mom<QH, 0, MODE, T, false>)
                          : (o32 ? k_collide_mom<QH, 1, MODE, T, true> : k_collide_mom<QH, 1, MODE, T, false>);
        Planes<T, T> pl{nullptr, (T*)c->g()};
        Timed tm(c, 2);
        hipLaunchKernelGGL(k, rows(c), dim3(NT), 0, c->stream, pl, (const T*)c->mom_buf(c->mom_cur),
                           (T*)c->mom_buf(1 - c->mom_cur), (const T*)c->phi(), (const T*)c->J(),
                           (const unsigned*)c->flags(par), c->cnt() + (1 - par), c->geo, physT(c),
                           c->nci_on() ? 1 : 0, macro, c->pa());
        if (MODE != MODE_DRY) c->mom_cur ^= 1;
        return;
      }
    }
    const bool o32 = off32(c);
    if constexpr (DIM == 3 && MODE == MODE_STEP) {
      if (par == 1 && row_collide(c)) {
        const bool wide = QH == 19 && sizeof(FS) == 4 && c->p.nx % 512 == 0;
        const bool one = wide && c->p.nx == 512;   // one cell per thread
        auto k = one ? (o32 ? k_collide_row<QH, T, FS, GS, true, 512, true>
                            : k_collide_row<QH, T, FS, GS, false, 512, true>)
                 : wide ? (o32 ? k_collide_row<QH, T, FS, GS, true, 512> : k_collide_row<QH, T, FS, GS, false, 512>)
                        : (o32 ? k_collide_row<QH, T, FS, GS, true, NT> : k_collide_row<QH, T, FS, GS, false, NT>);
        const unsigned lds = xrow_bytes<DIM, QH, FS, GS>(c->p.nx);
        Timed tm(c, 2);
        hipLaunchKernelGGL(k, dim3((unsigned)(c->p.ny * c->p.nz)), dim3(wide ? 512 : NT), lds, c->stream, planes(c), (const T*)c->phi(),
                           (const T*)c->J(), (const unsigned*)c->flags(par), c->cnt() + (1 - par), c->geo,
                           physT(c), c->nci_on() ? 1 : 0, c->fd() ? (T*)c->ua() : (T*)nullptr);
        return;
      }
    }
    auto k = par == 0
                 ? (o32 ? k_collide<DIM, QH, 0, MODE, T, FS, GS, true> : k_collide<DIM, QH, 0, MODE, T, FS, GS, false>)
                 : (o32 ? k_collide<DIM, QH, 1, MODE, T, FS, GS, true> : k_collide<DIM, QH, 1, MODE, T, FS, GS, false>);
    Timed tm(c, 2);
    hipLaunchKernelGGL(k, rows(c), dim3(NT), 0, c->stream, planes(c),
                       (const T*)c->phi(), (const T*)c->J(), (const unsigned*)c->flags(par),
                       c->cnt() + (1 - par), c->geo, physT(c), c->nci_on() ? 1 : 0, macro,
                       (MODE != MODE_DRY && c->fd()) ? (T*)c->ua() : (T*)nullptr, c->pa());
  }

  // Finite-difference phase field: phi of the next state into the other buffer.
  static void muscl_pass(lbm_ctx* c) {
    if (!c->fd()) return;
    const double kap = c->p.cac_compress ? 4.0 * c->p.mobility / c->p.width : 0.0;
    {
      Timed tm(c, 4);
      if constexpr (DIM == 3) {
        using M = MuslTile<T>;
        const int ntx = (c->p.nx + MZ_TX - 1) / MZ_TX, nty = (c->p.ny + M::TY - 1) / M::TY;
        const int nzc = (c->p.nz + MUSCL_ZRUN - 1) / MUSCL_ZRUN;
        hipLaunchKernelGGL((k_muscl3<QH, T>), dim3((unsigned)(ntx * nty * nzc)), dim3(M::NT), 0, c->stream,
                           (const T*)c->phi(), (T*)c->phi_next(), (const T*)c->ua(), c->geo,
                           (T)c->p.mobility, (T)kap, (T)c->p.eps_n, ntx, nty);
      } else {
        hipLaunchKernelGGL((k_muscl<DIM, QH, T>), rows(c), dim3(NT), 0, c->stream, (const T*)c->phi(),
                           (T*)c->phi_next(), (const T*)c->ua(), c->geo, (T)c->p.mobility, (T)kap,
                           (T)c->p.eps_n);
      }
    }
    c->phi_cur ^= 1;
  }

  static void diag_finish(lbm_ctx* c, int slot) {
    Timed tm(c, 3);
    hipLaunchKernelGGL((k_cc_init<DIM, T>), rows(c), dim3(NT), 0, c->stream, (const T*)c->phi(), c->geo,
                       c->dispersed, c->lab());
    hipLaunchKernelGGL((k_cc_merge<DIM, T>), rows(c), dim3(NT), 0, c->stream, (const T*)c->phi(), c->geo,
                       c->dispersed, c->lab());
    const int nd = (c->L.nblk + DIAG_PER - 1) / DIAG_PER;   // k_diag blocks
    hipLaunchKernelGGL((k_diag<DIM, T>), dim3((unsigned)nd), dim3(NT), 0, c->stream, (const T*)c->phi(), c->geo,
                       (const unsigned*)c->lab(), c->L.nblk, c->pb());
    const int chunk = (c->L.nblk + RED1 - 1) / RED1, chunkd = (nd + RED1 - 1) / RED1;
    hipLaunchKernelGGL(k_reduce_stage, dim3(RED1), dim3(NT), 0, c->stream, (const double*)c->pa(),
                       c->L.nblk, chunk, c->s1(0));
    hipLaunchKernelGGL(k_reduce_stage, dim3(RED1), dim3(NT), 0, c->stream, (const double*)c->pb(), nd, chunkd,
                       c->s1(1));
    hipLaunchKernelGGL(k_reduce, dim3(1), dim3(NT), 0, c->stream, (const double*)c->s1(0), RED1,
                       (const double*)c->s1(1), RED1,
                       (const unsigned*)(c->nci_on() ? c->cnt() + 2 : nullptr), c->red(slot));
  }

  static int step(lbm_ctx* c, int n) {
    const int K = c->p.diag_interval;
    for (int s = 0; s < n; ++s) {
      const int par = (int)(c->step & 1);
      phi_pass(c, par);
      nci_pass(c, par, nullptr, nullptr);
      const bool diag = K > 0 && (c->step % K) == 0;
      if (diag) {
        collide_pass<MODE_STEP_DIAG>(c, par, nullptr);
        const int slot = 1 + (c->hist_count % HIST);
        diag_finish(c, slot);
        c->hist_step[c->hist_count % HIST] = c->step;
        c->hist_count++;
      } else {
        collide_pass<MODE_STEP>(c, par, nullptr);
      }
      muscl_pass(c);
      c->step++;
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return c->fail(LBM_E_HIP, std::string("launch: ") + hipGetErrorString(e));
    return LBM_OK;
  }

  // Evaluate the current state without advancing it.  macro (device, may be
  // null) receives p*, rho, u, F; the reduction lands in red(0).
  static int evaluate(lbm_ctx* c, T* macro, int* chi, int* part) {
    const int par = (int)(c->step & 1);
    phi_pass(c, par);
    nci_pass(c, par, chi, part);
    collide_pass<MODE_DRY>(c, par, macro);
    diag_finish(c, 0);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return c->fail(LBM_E_HIP, std::string("launch: ") + hipGetErrorString(e));
    return LBM_OK;
  }

  static int init(lbm_ctx* c, const double* phi, const double* u, const double* ps) {
    const long long N = c->L.N, S = c->L.S;
    std::vector<T> hphi(N), hu((size_t)DIM * S, (T)0), hps(N);
    for (long long i = 0; i < N; ++i) {
      hphi[i] = (T)phi[i];
      hps[i] = (T)(ps ? ps[i] : c->p.pstar_ref);
      if (u)
        for (int a = 0; a < DIM; ++a) hu[(size_t)a * S + i] = (T)u[(size_t)a * N + i];
    }
    T *du = nullptr, *dps = nullptr;
    HIP_OR_FAIL(c, hipMalloc(&du, sizeof(T) * DIM * S));
    if (hipMalloc(&dps, sizeof(T) * S) != hipSuccess) {
      (void)hipFree(du);
      return c->fail(LBM_E_OOM, "temporary allocation failed");
    }
    int rc = LBM_OK;
    do {
      if (hipMemcpyAsync(c->phi(), hphi.data(), sizeof(T) * N, hipMemcpyHostToDevice, c->stream) ||
          hipMemcpyAsync(du, hu.data(), sizeof(T) * DIM * S, hipMemcpyHostToDevice, c->stream) ||
          hipMemcpyAsync(dps, hps.data(), sizeof(T) * N, hipMemcpyHostToDevice, c->stream)) {
        rc = c->fail(LBM_E_HIP, "host to device copy failed");
        break;
      }
      bool done = false;
      if constexpr (DIM == 3 && std::is_same<FS, T>::value && std::is_same<GS, T>::value) {
        if (c->mom()) {
          c->mom_cur = 0;
          hipLaunchKernelGGL((k_init_mom<QH, T>), rows(c), dim3(NT), 0, c->stream, (T*)c->mom_buf(0),
                             (T*)c->g(), (const T*)c->phi(), (const T*)du, (const T*)dps, c->geo, physT(c));
          done = true;
        }
      }
      if (!done)
        hipLaunchKernelGGL((k_init<DIM, QH, T, FS, GS>), rows(c), dim3(NT), 0, c->stream, (FS*)c->f(),
                           (GS*)c->g(), (const T*)c->phi(), (const T*)du, (const T*)dps, c->geo, physT(c));
      if (hipGetLastError() != hipSuccess || hipStreamSynchronize(c->stream) != hipSuccess)
        rc = c->fail(LBM_E_HIP, "initialisation kernel failed");
    } while (0);
    (void)hipFree(du);
    (void)hipFree(dps);
    return rc;
  }

  static int get_pop(lbm_ctx* c, int x0, int y0, int z0, int bx, int by, int bz, double* fo,
                     double* go) {
    const long long B = (long long)bx * by * bz;
    double *df = nullptr, *dg = nullptr;
    HIP_OR_FAIL(c, hipMalloc(&df, sizeof(double) * HydroQ<QH>::Q * B));
    if (hipMalloc(&dg, sizeof(double) * Phase<DIM>::Q * B) != hipSuccess) {
      (void)hipFree(df);
      return c->fail(LBM_E_OOM, "temporary allocation failed");
    }
    const int par = (int)(c->step & 1);
    bool done = false;
    if constexpr (DIM == 3 && std::is_same<FS, T>::value && std::is_same<GS, T>::value) {
      if (c->mom()) {
        auto k = par == 0 ? k_getpop_mom<QH, 0, T> : k_getpop_mom<QH, 1, T>;
        hipLaunchKernelGGL(k, dim3((unsigned)((B + NT - 1) / NT)), dim3(NT), 0, c->stream,
                           (const T*)c->mom_buf(c->mom_cur), (const T*)c->g(), c->geo, x0, y0, z0, bx, by, bz,
                           df, dg);
        done = true;
      }
    }
    if (!done) {
      auto k = par == 0 ? k_getpop<DIM, QH, 0, T, FS, GS> : k_getpop<DIM, QH, 1, T, FS, GS>;
      hipLaunchKernelGGL(k, dim3((unsigned)((B + NT - 1) / NT)), dim3(NT), 0, c->stream,
                         (const FS*)c->f(), (const GS*)c->g(), c->geo, physT(c), x0, y0, z0, bx, by, bz,
                         df, dg);
    }
    int rc = LBM_OK;
    if (hipStreamSynchronize(c->stream) != hipSuccess ||
        (fo && hipMemcpy(fo, df, sizeof(double) * HydroQ<QH>::Q * B, hipMemcpyDeviceToHost)) ||
        (go && hipMemcpy(go, dg, sizeof(double) * Phase<DIM>::Q * B, hipMemcpyDeviceToHost)))
      rc = c->fail(LBM_E_HIP, "population read-back failed");
    (void)hipFree(df);
    (void)hipFree(dg);
    return rc;
  }

  static int set_pop(lbm_ctx* c, const double* fi, const double* gi) {
    const long long N = c->L.N;
    double *df = nullptr, *dg = nullptr;
    HIP_OR_FAIL(c, hipMalloc(&df, sizeof(double) * HydroQ<QH>::Q * N));
    if (hipMalloc(&dg, sizeof(double) * Phase<DIM>::Q * N) != hipSuccess) {
      (void)hipFree(df);
      return c->fail(LBM_E_OOM, "temporary allocation failed");
    }
    int rc = LBM_OK;
    if (hipMemcpy(df, fi, sizeof(double) * HydroQ<QH>::Q * N, hipMemcpyHostToDevice) ||
        hipMemcpy(dg, gi, sizeof(double) * Phase<DIM>::Q * N, hipMemcpyHostToDevice)) {
      rc = c->fail(LBM_E_HIP, "host to device copy failed");
    } else {
      hipLaunchKernelGGL((k_setpop<DIM, QH, T, FS, GS>), dim3((unsigned)((N + NT - 1) / NT)), dim3(NT), 0,
                         c->stream, (FS*)c->f(), (GS*)c->g(), c->geo, physT(c), df, dg);
      if (hipStreamSynchronize(c->stream) != hipSuccess) rc = c->fail(LBM_E_HIP, "set kernel failed");
    }
    (void)hipFree(df);
    (void)hipFree(dg);
    return rc;
  }

  // which: 0 p*, 1 rho, 2 u, 3 F
  static int get_macro(lbm_ctx* c, int which, double* out) {
    T* macro = nullptr;
    const long long S = c->L.S;
    HIP_OR_FAIL(c, hipMalloc(&macro, sizeof(T) * (2 + 2 * DIM) * S));
    int rc = evaluate(c, macro, nullptr, nullptr);
    if (rc == LBM_OK) {
      const long long first = which == 0 ? 0 : (which == 1 ? 1 : (which == 2 ? 2 : 2 + DIM));
      const long long comps = which <= 1 ? 1 : DIM;
      rc = copy_field_to_host<T>(c, macro + first * S, comps, out);
    }
    (void)hipFree(macro);
    return rc;
  }

  // Swarm statistics of the current state (stats.hpp).
  static int curvature_hist(lbm_ctx* c, double q_band, double kmin, double kmax, int nbins, long* out) {
    const int par = (int)(c->step & 1);
    phi_pass(c, par);
    T* n = nullptr;
    unsigned long long* dc = nullptr;
    HIP_OR_FAIL(c, hipMalloc(&n, sizeof(T) * DIM * c->L.S));
    if (hipMalloc(&dc, sizeof(unsigned long long) * (nbins + 2)) != hipSuccess) {
      (void)hipFree(n);
      return c->fail(LBM_E_OOM, "temporary allocation failed");
    }
    int rc = LBM_OK;
    std::vector<unsigned long long> h((size_t)nbins + 2);
    const T sgn = c->dispersed ? (T)-1 : (T)1;
    if (hipMemsetAsync(dc, 0, sizeof(unsigned long long) * (nbins + 2), c->stream) != hipSuccess) {
      rc = c->fail(LBM_E_HIP, "memset failed");
    } else {
      hipLaunchKernelGGL((k_normal<DIM, QH, T>), rows(c), dim3(NT), 0, c->stream, (const T*)c->phi(), n, c->geo,
                         sgn, (T)c->p.eps_n);
      hipLaunchKernelGGL((k_curv_hist<DIM, QH, T>), rows(c), dim3(NT), 0, c->stream, (const T*)c->phi(),
                         (const T*)n, c->geo, (T)q_band, kmin, kmax, nbins, dc);
      if (hipGetLastError() != hipSuccess || hipStreamSynchronize(c->stream) != hipSuccess ||
          hipMemcpy(h.data(), dc, sizeof(unsigned long long) * (nbins + 2), hipMemcpyDeviceToHost) != hipSuccess)
        rc = c->fail(LBM_E_HIP, "curvature histogram failed");
    }
    for (int b = 0; rc == LBM_OK && b < nbins + 2; ++b) out[b] = (long)h[b];
    (void)hipFree(n);
    (void)hipFree(dc);
    return rc;
  }

  static int component_volumes(lbm_ctx* c, long* out, long max, long* count) {
    const int par = (int)(c->step & 1);
    phi_pass(c, par);
    const long long N = c->L.N;
    const unsigned cap = (unsigned)std::min<long>(max, (long)N);
    unsigned *vol = nullptr, *lst = nullptr;
    HIP_OR_FAIL(c, hipMalloc(&vol, sizeof(unsigned) * (N + 1 + (long long)cap)));
    lst = vol + N + 1;   // [N] is the component counter, then the list
    int rc = LBM_OK;
    unsigned n = 0;
    std::vector<unsigned> h(cap);
    if (hipMemsetAsync(vol, 0, sizeof(unsigned) * (N + 1), c->stream) != hipSuccess) {
      rc = c->fail(LBM_E_HIP, "memset failed");
    } else {
      hipLaunchKernelGGL((k_cc_init<DIM, T>), rows(c), dim3(NT), 0, c->stream, (const T*)c->phi(), c->geo,
                         c->dispersed, c->lab());
      hipLaunchKernelGGL((k_cc_merge<DIM, T>), rows(c), dim3(NT), 0, c->stream, (const T*)c->phi(), c->geo,
                       c->dispersed, c->lab());
      hipLaunchKernelGGL(k_cc_volume, rows(c), dim3(NT), 0, c->stream, c->geo, (const unsigned*)c->lab(), vol);
      hipLaunchKernelGGL(k_cc_list, rows(c), dim3(NT), 0, c->stream, c->geo, (const unsigned*)c->lab(),
                         (const unsigned*)vol, lst, cap, vol + N);
      if (hipGetLastError() != hipSuccess || hipStreamSynchronize(c->stream) != hipSuccess ||
          hipMemcpy(&n, vol + N, sizeof(unsigned), hipMemcpyDeviceToHost) != hipSuccess ||
          (cap && hipMemcpy(h.data(), lst, sizeof(unsigned) * cap, hipMemcpyDeviceToHost) != hipSuccess))
        rc = c->fail(LBM_E_HIP, "component volumes failed");
    }
    if (rc == LBM_OK) {
      const unsigned m = std::min(n, cap);
      std::sort(h.begin(), h.begin() + m, [](unsigned a, unsigned b) { return a > b; });
      for (unsigned k = 0; k < m; ++k) out[k] = (long)h[k];
      *count = (long)n;
    }
    (void)hipFree(vol);
    return rc;
  }

  static int get_phi(lbm_ctx* c, double* out) {
    const int par = (int)(c->step & 1);
    phi_pass(c, par);
    return copy_field_to_host<T>(c, (const T*)c->phi(), 1, out);
  }

  static int get_nci(lbm_ctx* c, int* chi, int* part, double* J) {
    const long long N = c->L.N;
    int *dchi = nullptr, *dpart = nullptr;
    HIP_OR_FAIL(c, hipMalloc(&dchi, sizeof(int) * N));
    if (hipMalloc(&dpart, sizeof(int) * 3 * N) != hipSuccess) {
      (void)hipFree(dchi);
      return c->fail(LBM_E_OOM, "temporary allocation failed");
    }
    int rc = LBM_OK;
    (void)hipMemsetAsync(dchi, 0, sizeof(int) * N, c->stream);
    (void)hipMemsetAsync(dpart, 0, sizeof(int) * 3 * N, c->stream);
    (void)hipMemsetAsync(c->J(), 0, sizeof(T) * DIM * c->L.S, c->stream);
    const int par = (int)(c->step & 1);
    phi_pass(c, par);
    nci_pass(c, par, dchi, dpart);
    if (hipStreamSynchronize(c->stream) != hipSuccess) rc = c->fail(LBM_E_HIP, "near-contact pass failed");
    if (rc == LBM_OK && chi && hipMemcpy(chi, dchi, sizeof(int) * N, hipMemcpyDeviceToHost)) rc = LBM_E_HIP;
    if (rc == LBM_OK && part && hipMemcpy(part, dpart, sizeof(int) * 3 * N, hipMemcpyDeviceToHost)) rc = LBM_E_HIP;
    if (rc == LBM_OK && J) rc = copy_field_to_host<T>(c, (const T*)c->J(), DIM, J);
    (void)hipFree(dchi);
    (void)hipFree(dpart);
    return rc;
  }

  static int diagnostics(lbm_ctx* c, lbm_diag* out) {
    int rc = evaluate(c, nullptr, nullptr, nullptr);
    if (rc != LBM_OK) return rc;
    double r[2 * NPART];
    HIP_OR_FAIL(c, hipMemcpyAsync(r, c->red(0), sizeof(r), hipMemcpyDeviceToHost, c->stream));
    HIP_OR_FAIL(c, hipStreamSynchronize(c->stream));
    fill_diag(r, c->step, out);
    return LBM_OK;
  }

  // ---- serving: several lattices advanced by multi-domain launches
  using JobT = Job<T, FS, GS>;

  static void batch_launch(hipStream_t st, const JobT* dj, int nj, int blocks, int pblocks, int s, bool o32) {
    hipLaunchKernelGGL((k_phi_multi<DIM, T, FS, GS>), dim3((unsigned)pblocks), dim3(NT), 0, st, dj, nj, s);
    hipLaunchKernelGGL((k_nci_multi<DIM, QH, T, FS, GS>), dim3(NCI_GRID), dim3(NT_NCI), 0, st, dj, nj, s);
    if (o32)
      hipLaunchKernelGGL((k_collide_multi<DIM, QH, T, FS, GS, true>), dim3((unsigned)blocks), dim3(NT), 0, st,
                         dj, nj, s);
    else
      hipLaunchKernelGGL((k_collide_multi<DIM, QH, T, FS, GS, false>), dim3((unsigned)blocks), dim3(NT), 0,
                         st, dj, nj, s);
  }

  // Table entry of one lattice whose blocks start at blk0 of the batch grid
  // (and at pblk0 of the phi pass's grid).
  static JobT job_entry(lbm_ctx* c, int blk0, int pblk0) {
    JobT jb{};
    jb.pl = planes(c);
    jb.phi = (T*)c->phi();
    jb.J = (T*)c->J();
    for (int k = 0; k < 2; ++k) {
      jb.flags[k] = c->flags(k);
      jb.list[k] = c->list(k);
    }
    jb.cnt = c->cnt();
    jb.geo = c->geo;
    jb.pp = physT(c);
    jb.np = c->nci;
    jb.nci_on = c->nci_on() ? 1 : 0;
    jb.q_th = (T)c->p.q_th;
    jb.blk0 = blk0;
    jb.nblk = c->L.nblk;
    jb.pblk0 = pblk0;
    jb.pnblk = (c->L.nblk + PHI_PER - 1) / PHI_PER;
    jb.step = c->step;
    return jb;
  }

  // The same steps as batch() with the job table in the device's static
  // array: no allocation, no graph; the table is written on the first context's
  // stream by small kernels (entries passed by value) and the call waits for
  // its steps before returning.
  static int batch_noalloc(lbm_ctx* const* cs, int count, int n, JobT* table) {
    static_assert(sizeof(JobT) <= STATIC_JOB_BYTES, "job table entry larger than its static slot");
    constexpr int K = 2048 / sizeof(JobT) > 64 ? 64 : (int)(2048 / sizeof(JobT));
    static_assert(K >= 1, "job table entry too large for kernel arguments");
    lbm_ctx* c0 = cs[0];
    hipStream_t st = c0->stream;
    for (int i = 1; i < count; ++i) HIP_OR_FAIL(c0, hipStreamSynchronize(cs[i]->stream));
    int blocks = 0, pblocks = 0;
    bool o32 = true;
    for (int i0 = 0; i0 < count; i0 += K) {
      JobChunk<JobT, K> chunk{};
      const int m = std::min(K, count - i0);
      for (int k = 0; k < m; ++k) {
        chunk.j[k] = job_entry(cs[i0 + k], blocks, pblocks);
        blocks += cs[i0 + k]->L.nblk;
        pblocks += chunk.j[k].pnblk;
        o32 = o32 && off32(cs[i0 + k]);
      }
      hipLaunchKernelGGL((k_put_jobs<JobT, K>), dim3(1), dim3(64), 0, st, table + i0, chunk, m);
    }
    for (int sidx = 0; sidx < n; ++sidx) batch_launch(st, table, count, blocks, pblocks, sidx, o32);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return c0->fail(LBM_E_HIP, std::string("batch launch: ") + hipGetErrorString(e));
    HIP_OR_FAIL(c0, hipStreamSynchronize(st));
    for (int i = 0; i < count; ++i) cs[i]->step += n;
    return LBM_OK;
  }

  static int batch(lbm_ctx* const* cs, int count, int n) {
    lbm_ctx* c0 = cs[0];
    hipStream_t st = c0->stream;
    for (int i = 1; i < count; ++i) HIP_OR_FAIL(c0, hipStreamSynchronize(cs[i]->stream));
    // find or create the cached batch of this ordered set of contexts
    Batch* B = nullptr;
    for (Batch* b : batches())
      if ((int)b->ctxs.size() == count && std::equal(b->ctxs.begin(), b->ctxs.end(), cs)) B = b;
    if (!B) {
      if ((int)batches().size() >= BATCH_CACHE) {
        delete batches().front();
        batches().erase(batches().begin());
      }
      B = new Batch();
      B->ctxs.assign(cs, cs + count);
      B->bytes = sizeof(JobT) * (size_t)count;
      if (hipMalloc(&B->djobs, B->bytes) != hipSuccess || hipHostMalloc(&B->hjobs, B->bytes) != hipSuccess ||
          hipEventCreateWithFlags(&B->done, hipEventDisableTiming) != hipSuccess ||
          hipEventCreateWithFlags(&B->copied, hipEventDisableTiming) != hipSuccess) {
        delete B;
        return c0->fail(LBM_E_OOM, "batch table allocation failed");
      }
      batches().push_back(B);
    }
    // the job table of this call; the pinned mirror is rewritten only once the
    // previous call's upload from it has executed
    if (B->used) HIP_OR_FAIL(c0, hipEventSynchronize(B->copied));
    JobT* hj = (JobT*)B->hjobs;
    int blocks = 0, pblocks = 0;
    bool o32 = true;
    for (int i = 0; i < count; ++i) {
      hj[i] = job_entry(cs[i], blocks, pblocks);
      blocks += cs[i]->L.nblk;
      pblocks += hj[i].pnblk;
      o32 = o32 && off32(cs[i]);
    }
    HIP_OR_FAIL(c0, hipMemcpyAsync(B->djobs, B->hjobs, B->bytes, hipMemcpyHostToDevice, st));
    HIP_OR_FAIL(c0, hipEventRecord(B->copied, st));
    B->used = true;
    const JobT* dj = (const JobT*)B->djobs;
    const int full = n / BATCH_R, rem = n % BATCH_R;
    if (full > 0) {
      if (!B->exec || B->total_blocks != blocks || B->o32 != o32) {
        if (B->exec) (void)hipGraphExecDestroy(B->exec);
        if (B->graph) (void)hipGraphDestroy(B->graph);
        B->exec = nullptr;
        B->graph = nullptr;
        HIP_OR_FAIL(c0, hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
        for (int sidx = 0; sidx < BATCH_R; ++sidx) batch_launch(st, dj, count, blocks, pblocks, sidx, o32);
        hipLaunchKernelGGL((k_advance<T, FS, GS>), dim3((count + 63) / 64), dim3(64), 0, st,
                           (JobT*)B->djobs, count, BATCH_R);
        HIP_OR_FAIL(c0, hipStreamEndCapture(st, &B->graph));
        HIP_OR_FAIL(c0, hipGraphInstantiate(&B->exec, B->graph, nullptr, nullptr, 0));
        B->total_blocks = blocks;
        B->o32 = o32;
      }
      for (int k = 0; k < full; ++k) HIP_OR_FAIL(c0, hipGraphLaunch(B->exec, st));
    }
    for (int sidx = 0; sidx < rem; ++sidx) batch_launch(st, dj, count, blocks, pblocks, sidx, o32);
    if (rem)
      hipLaunchKernelGGL((k_advance<T, FS, GS>), dim3((count + 63) / 64), dim3(64), 0, st,
                         (JobT*)B->djobs, count, rem);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return c0->fail(LBM_E_HIP, std::string("batch launch: ") + hipGetErrorString(e));
    for (int i = 0; i < count; ++i) cs[i]->step += n;
    // later work on the other contexts' streams waits for the batch
    HIP_OR_FAIL(c0, hipEventRecord(B->done, st));
    for (int i = 1; i < count; ++i) HIP_OR_FAIL(c0, hipStreamWaitEvent(cs[i]->stream, B->done, 0));
    return LBM_OK;
  }
};

// Dispatch a functor over the (lattice, precision) combinations that are built.
template <int DIM, int QH, typename Fn>
int dispatch_prec(int pr, Fn&& fn) {
  if (pr == LBM_FP64) return fn(Engine<DIM, QH, double, double, double>{});
  if (pr == LBM_FP32) return fn(Engine<DIM, QH, float, float, float>{});
  if (pr == LBM_FP32_F16STORE) return fn(Engine<DIM, QH, float, __half, float>{});
  if (pr == LBM_FP32_BF16STORE) return fn(Engine<DIM, QH, float, __hip_bfloat16, float>{});
  return LBM_E_UNSUPPORTED;
}
template <typename Fn>
int dispatch(const lbm_ctx* c, Fn&& fn) {
  const int pr = c->p.precision;
  if (c->p.dim == 2) return dispatch_prec<2, 9>(pr, fn);
  if (q_hydro(&c->p) == 27) return dispatch_prec<3, 27>(pr, fn);
  return dispatch_prec<3, 19>(pr, fn);
}

void reset_nci_state(lbm_ctx* c) {
  const Layout& L = c->L;
  (void)hipMemsetAsync(c->ws + L.off_flags, 0, 2 * (size_t)L.ntiles * 4, c->stream);
  (void)hipMemsetAsync(c->ws + L.off_cnt, 0, 64, c->stream);
  (void)hipMemsetAsync(c->J(), 0, (size_t)c->p.dim * L.S * real_size(c->p.precision), c->stream);
}

// Mixture and forcing constants of the current parameters (Sec. 2.1).
void set_phys(lbm_ctx* c, double mean_phi) {
  const lbm_params& p = c->p;
  const double cs2 = 1.0 / 3.0;
  const double rho_l = 1.0, rho_g = 1.0 / p.density_ratio;
  const double nu_l = cs2 * (p.tau - 0.5), nu_g = p.visc_ratio * nu_l;
  Phys& P = c->phys;
  P.rho_g = rho_g;
  P.drho = rho_l - rho_g;
  P.mu_a = rho_g * nu_g;
  P.mu_b = rho_l * nu_l - rho_g * nu_g;
  P.beta4 = 4.0 * 12.0 * p.sigma / p.width;
  P.kappa = 1.5 * p.sigma * p.width;
  P.rho_mean = rho_g + (rho_l - rho_g) * mean_phi;
  for (int a = 0; a < 3; ++a) P.g[a] = a < p.dim ? p.body_force[a] : 0.0;
  P.kc = p.cac_compress ? p.mobility * 4.0 / p.width : 0.0;
  const double cs2_phi = p.dim == 2 ? 1.0 / 3.0 : 0.25;
  P.inv_tau_phi = 1.0 / (0.5 + p.mobility / cs2_phi);
  P.pstar_ref = p.pstar_ref;
  P.eps_n = p.eps_n;
}

}  // namespace

// ===========================================================================
// C ABI
// ===========================================================================

extern "C" {

void lbm_default_params(lbm_params* p) {
  if (!p) return;
  std::memset(p, 0, sizeof(*p));
  p->dim = 2;
  p->nx = 128;
  p->ny = 128;
  p->nz = 1;
  p->precision = LBM_FP64;
  p->tau = 1.0;
  p->visc_ratio = 1.0;
  p->mobility = 0.1;
  p->width = 4.0;
  p->sigma = 1e-3;
  p->density_ratio = 1.0;
  p->a_rep = 1e-3;
  p->nci_window = 3;
  p->q_th = 0.125;
  p->eta = 0.1;
  p->cos_opp = -0.8;
  p->h0 = 1.0;
  p->p_exp = 4.0;
  p->eps_n = 1e-12;
  p->eps_q = 1e-6;
  p->tie_eps = 1e-6;
  p->rep_orient = 0;
  p->dispersed = -1;
  p->cac_compress = 1;
  p->diag_interval = 0;
  p->pstar_ref = 0.0;
}

size_t lbm_workspace_bytes(const lbm_params* p) {
  if (!valid_params(p, nullptr)) return 0;
  return make_layout(p).total;
}

int lbm_create(const lbm_params* p, void* dev_workspace, size_t ws_bytes, void* hip_stream,
               lbm_ctx** out) {
  if (!out) return LBM_E_INVALID;
  *out = nullptr;
  std::string why;
  if (!valid_params(p, &why)) {
    g_create_error = why;
    return LBM_E_INVALID;
  }
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) {
    g_create_error = "no HIP device";
    return LBM_E_HIP;
  }
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, dev) != hipSuccess) {
    g_create_error = "hipGetDeviceProperties failed";
    return LBM_E_HIP;
  }
  if (!supported(p, &why)) {
    g_create_error = why;
    return LBM_E_UNSUPPORTED;
  }
  if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0) {
    g_create_error = std::string("this library is built for gfx950, device is ") + prop.gcnArchName;
    return LBM_E_UNSUPPORTED;
  }
  lbm_ctx* c = new lbm_ctx();
  c->p = *p;
  c->dev = dev;
  c->L = make_layout(p);
  if (dev_workspace) {
    if (ws_bytes < c->L.total || ((uintptr_t)dev_workspace & 255)) {
      g_create_error = "workspace too small or not 256-byte aligned";
      delete c;
      return LBM_E_OOM;
    }
    c->ws = (char*)dev_workspace;
  } else {
    if (hipMalloc((void**)&c->ws, c->L.total) != hipSuccess) {
      g_create_error = "device allocation of the workspace failed";
      delete c;
      return LBM_E_OOM;
    }
    c->own_ws = true;
  }
  if (hip_stream) {
    c->stream = (hipStream_t)hip_stream;
  } else {
    if (hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking) != hipSuccess) {
      if (c->own_ws) (void)hipFree(c->ws);
      delete c;
      g_create_error = "stream creation failed";
      return LBM_E_HIP;
    }
    c->own_stream = true;
  }
  Geo& G = c->geo;
  G.nx = p->nx;
  G.ny = p->ny;
  G.nz = p->nz;
  G.bxs = c->L.bxs;
  G.nbx = (p->nx + (1 << G.bxs) - 1) >> G.bxs;
  G.nby = (p->ny + (NT >> G.bxs) - 1) / (NT >> G.bxs);
  G.S = c->L.S;
  G.ntx = c->L.ntx;
  G.nty = c->L.nty;
  G.ntz = c->L.ntz;
  G.rs = c->L.rs;
  G.qc = c->L.qc;
  NciP& A = c->nci;
  A.a_rep = p->a_rep;
  A.q_th = p->q_th;
  A.eta = p->eta;
  A.cos_opp = p->cos_opp;
  A.h0 = p->h0;
  A.p_exp = p->p_exp;
  A.eps_n = p->eps_n;
  A.eps_q = p->eps_q;
  A.tie_eps = p->tie_eps;
  A.width = p->width;
  A.w = p->nci_window;
  A.orient = p->rep_orient;
  set_phys(c, 0.0);
  (void)hipMemsetAsync(c->ws, 0, c->L.total, c->stream);
  if (hipStreamSynchronize(c->stream) != hipSuccess) {
    g_create_error = "workspace clear failed";
    lbm_destroy(c);
    return LBM_E_HIP;
  }
  *out = c;
  return LBM_OK;
}

void lbm_destroy(lbm_ctx* c) {
  if (!c) return;
  if (c->stream) (void)hipStreamSynchronize(c->stream);
  forget_batches_of(c);
  for (hipEvent_t e : c->ev) (void)hipEventDestroy(e);
  if (c->own_ws && c->ws) (void)hipFree(c->ws);
  if (c->own_stream && c->stream) (void)hipStreamDestroy(c->stream);
  delete c;
}

const char* lbm_last_error(const lbm_ctx* c) { return c ? c->err.c_str() : g_create_error.c_str(); }

int lbm_init_fields(lbm_ctx* c, const double* phi, const double* u, const double* pstar) {
  if (!c || !phi) return c ? c->fail(LBM_E_INVALID, "phi is required") : LBM_E_INVALID;
  double acc = 0.0;
  for (long long i = 0; i < c->L.N; ++i) acc += phi[i];
  const double mean_phi = acc / (double)c->L.N;
  set_phys(c, mean_phi);
  c->dispersed = c->p.dispersed >= 0 ? c->p.dispersed : (mean_phi < 0.5 ? 1 : 0);
  reset_nci_state(c);
  c->phi_cur = 0;
  const int rc = dispatch(c, [&](auto E) { return decltype(E)::init(c, phi, u, pstar); });
  if (rc != LBM_OK) return rc;
  c->step = 0;
  c->hist_count = 0;
  c->initialised = true;
  return LBM_OK;
}

int lbm_step(lbm_ctx* c, int n) {
  if (!c) return LBM_E_INVALID;
  if (n < 0) return c->fail(LBM_E_INVALID, "negative step count");
  if (!c->initialised) return c->fail(LBM_E_STATE, "lbm_step before lbm_init_fields");
  return dispatch(c, [&](auto E) { return decltype(E)::step(c, n); });
}

long lbm_step_count(const lbm_ctx* c) { return c ? c->step : -1; }

int lbm_diag_history(lbm_ctx* c, lbm_diag* out, int max) {
  if (!c || (!out && max > 0)) return LBM_E_INVALID;
  HIP_OR_FAIL(c, hipStreamSynchronize(c->stream));
  const int have = std::min(c->hist_count, HIST);
  std::vector<double> buf((size_t)(HIST + 1) * 2 * NPART);
  HIP_OR_FAIL(c, hipMemcpy(buf.data(), c->red(0), buf.size() * 8, hipMemcpyDeviceToHost));
  int k = 0;
  for (int j = std::max(0, c->hist_count - HIST); j < c->hist_count && k < max; ++j, ++k) {
    fill_diag(&buf[(size_t)(1 + (j % HIST)) * 2 * NPART], c->hist_step[j % HIST], &out[k]);
  }
  (void)have;
  return k;
}

int lbm_sync(lbm_ctx* c) {
  if (!c) return LBM_E_INVALID;
  HIP_OR_FAIL(c, hipStreamSynchronize(c->stream));
  if (c->p.diag_interval > 0 && c->hist_count > 0) {
    std::vector<lbm_diag> h(HIST);
    const int n = lbm_diag_history(c, h.data(), HIST);
    for (int i = 0; i < n; ++i)
      if (!h[i].finite) return c->fail(LBM_E_DIVERGED, "non-finite value at step " + std::to_string(h[i].step));
  }
  return LBM_OK;
}

#define NEED_INIT(c)                                                              \
  do {                                                                            \
    if (!(c)) return LBM_E_INVALID;                                               \
    if (!(c)->initialised) return (c)->fail(LBM_E_STATE, "context not initialised"); \
  } while (0)

int lbm_get_phi(lbm_ctx* c, double* out) {
  NEED_INIT(c);
  if (!out) return c->fail(LBM_E_INVALID, "null output");
  return dispatch(c, [&](auto E) { return decltype(E)::get_phi(c, out); });
}

int lbm_curvature_histogram(lbm_ctx* c, double q_band, double kmin, double kmax, int nbins, long* counts) {
  NEED_INIT(c);
  if (!counts) return c->fail(LBM_E_INVALID, "null output");
  if (nbins < 1 || nbins > STATS_MAX_BINS) return c->fail(LBM_E_INVALID, "nbins must be in [1, 4096]");
  if (!(kmax > kmin) || !(q_band > 0.0) || !(q_band <= 0.25))
    return c->fail(LBM_E_INVALID, "need kmax > kmin and 0 < q_band <= 1/4");
  return dispatch(c, [&](auto E) { return decltype(E)::curvature_hist(c, q_band, kmin, kmax, nbins, counts); });
}

int lbm_component_volumes(lbm_ctx* c, long* volumes, long max, long* count) {
  NEED_INIT(c);
  if (!count || max < 0 || (max > 0 && !volumes)) return c->fail(LBM_E_INVALID, "bad output");
  return dispatch(c, [&](auto E) { return decltype(E)::component_volumes(c, volumes, max, count); });
}

int lbm_get_pstar(lbm_ctx* c, double* out) {
  NEED_INIT(c);
  if (!out) return c->fail(LBM_E_INVALID, "null output");
  return dispatch(c, [&](auto E) { return decltype(E)::get_macro(c, 0, out); });
}

int lbm_get_rho(lbm_ctx* c, double* out) {
  NEED_INIT(c);
  if (!out) return c->fail(LBM_E_INVALID, "null output");
  return dispatch(c, [&](auto E) { return decltype(E)::get_macro(c, 1, out); });
}

int lbm_get_u(lbm_ctx* c, double* out) {
  NEED_INIT(c);
  if (!out) return c->fail(LBM_E_INVALID, "null output");
  return dispatch(c, [&](auto E) { return decltype(E)::get_macro(c, 2, out); });
}

int lbm_get_force(lbm_ctx* c, double* out) {
  NEED_INIT(c);
  if (!out) return c->fail(LBM_E_INVALID, "null output");
  return dispatch(c, [&](auto E) { return decltype(E)::get_macro(c, 3, out); });
}

int lbm_get_nci(lbm_ctx* c, int* chi, int* partner, double* J) {
  NEED_INIT(c);
  return dispatch(c, [&](auto E) { return decltype(E)::get_nci(c, chi, partner, J); });
}

int lbm_diagnostics(lbm_ctx* c, lbm_diag* out) {
  NEED_INIT(c);
  if (!out) return c->fail(LBM_E_INVALID, "null output");
  return dispatch(c, [&](auto E) { return decltype(E)::diagnostics(c, out); });
}

int lbm_lattice(int dim, int which, int* c) {
  if (dim != 2 && dim != 3) return LBM_E_INVALID;
  if (which < 0 || which > 2 || (which == 2 && dim != 3)) return LBM_E_INVALID;
  const int q = which == 0 ? q_hydro(dim) : (which == 1 ? q_phase(dim) : 27);
  if (c) {
    for (int i = 0; i < q; ++i) {
      if (which == 2) {
        c[3 * i] = HydroQ<27>::cx[i];
        c[3 * i + 1] = HydroQ<27>::cy[i];
        c[3 * i + 2] = HydroQ<27>::cz[i];
      } else if (dim == 2) {
        c[3 * i] = Hydro<2>::cx[i];
        c[3 * i + 1] = Hydro<2>::cy[i];
        c[3 * i + 2] = 0;
      } else if (which == 0) {
        c[3 * i] = Hydro<3>::cx[i];
        c[3 * i + 1] = Hydro<3>::cy[i];
        c[3 * i + 2] = Hydro<3>::cz[i];
      } else {
        c[3 * i] = Phase<3>::cx[i];
        c[3 * i + 1] = Phase<3>::cy[i];
        c[3 * i + 2] = Phase<3>::cz[i];
      }
    }
  }
  return q;
}

int lbm_get_populations(lbm_ctx* c, int x0, int y0, int z0, int bx, int by, int bz, double* f,
                        double* g) {
  NEED_INIT(c);
  if (bx < 1 || by < 1 || bz < 1 || (c->p.dim == 2 && bz != 1))
    return c->fail(LBM_E_INVALID, "bad box");
  return dispatch(c, [&](auto E) { return decltype(E)::get_pop(c, x0, y0, z0, bx, by, bz, f, g); });
}

int lbm_set_populations(lbm_ctx* c, const double* f, const double* g) {
  if (!c) return LBM_E_INVALID;
  if (!f || !g) return c->fail(LBM_E_INVALID, "null populations");
  if (c->fd())
    return c->fail(LBM_E_UNSUPPORTED, "the finite-difference phase field has no populations g to set");
  if (c->mom())
    return c->fail(LBM_E_UNSUPPORTED,
                   "moment storage keeps post-collision coefficients, which arbitrary populations need not have");
  // mean phi (for the buoyancy reference) from the phase-field populations
  const long long N = c->L.N;
  const int qg = q_phase(c->p.dim);
  double acc = 0.0;
  for (long long i = 0; i < N; ++i) {
    double s = 0.0;
    for (int k = 0; k < qg; ++k) s += g[(size_t)k * N + i];
    acc += s;
  }
  const double mean_phi = acc / (double)N;
  set_phys(c, mean_phi);
  c->dispersed = c->p.dispersed >= 0 ? c->p.dispersed : (mean_phi < 0.5 ? 1 : 0);
  reset_nci_state(c);
  const int rc = dispatch(c, [&](auto E) { return decltype(E)::set_pop(c, f, g); });
  if (rc != LBM_OK) return rc;
  c->step = 0;
  c->hist_count = 0;
  c->initialised = true;
  return LBM_OK;
}

// Raw state: header {magic, format version, step, rho_mean, dispersed, box,
// precision, lattice, phase-field solver} + f + g as stored (+ phi with the
// finite-difference phase field).
namespace {
struct StateHeader {
  unsigned long long magic;
  long long version;
  long long step;
  double rho_mean;
  long long dispersed;
  long long dim, nx, ny, nz, precision, hydro_q, cac_solver, hydro_store, store_cur;
};
constexpr unsigned long long STATE_MAGIC = 0x4c424d5354415445ULL;  // "LBMSTATE"
constexpr long long STATE_VERSION = 3;
StateHeader state_header(const lbm_ctx* c) {
  return StateHeader{STATE_MAGIC, STATE_VERSION, c->step, c->phys.rho_mean, c->dispersed, c->p.dim,
                     c->p.nx, c->p.ny, c->p.nz, c->p.precision, q_hydro(&c->p), c->p.cac_solver,
                     c->p.hydro_store, c->mom_cur};
}
size_t pop_bytes(const lbm_ctx* c) {
  return c->L.off_phi;  // f and g are the first two regions of the workspace
}
// the finite-difference phase field keeps phi itself as state
size_t phi_state_bytes(const lbm_ctx* c) {
  return c->fd() ? (size_t)c->L.N * real_size(c->p.precision) : 0;
}
}  // namespace

size_t lbm_state_bytes(const lbm_ctx* c) {
  return c ? sizeof(StateHeader) + pop_bytes(c) + phi_state_bytes(c) : 0;
}

int lbm_save_state(lbm_ctx* c, void* buf, size_t bytes) {
  NEED_INIT(c);
  if (!buf || bytes < lbm_state_bytes(c)) return c->fail(LBM_E_INVALID, "state buffer too small");
  const StateHeader h = state_header(c);
  std::memcpy(buf, &h, sizeof(h));
  HIP_OR_FAIL(c, hipStreamSynchronize(c->stream));
  HIP_OR_FAIL(c, hipMemcpy((char*)buf + sizeof(h), c->ws, pop_bytes(c), hipMemcpyDeviceToHost));
  if (c->fd())
    HIP_OR_FAIL(c, hipMemcpy((char*)buf + sizeof(h) + pop_bytes(c), c->phi(), phi_state_bytes(c),
                             hipMemcpyDeviceToHost));
  return LBM_OK;
}

int lbm_load_state(lbm_ctx* c, const void* buf, size_t bytes) {
  if (!c) return LBM_E_INVALID;
  if (!buf || bytes != lbm_state_bytes(c))
    return c->fail(LBM_E_INVALID, "state size does not match this context");
  StateHeader h;
  std::memcpy(&h, buf, sizeof(h));
  const StateHeader want = state_header(c);
  if (h.magic != STATE_MAGIC || h.version != STATE_VERSION)
    return c->fail(LBM_E_INVALID, "not a state of this library version");
  if (h.dim != want.dim || h.nx != want.nx || h.ny != want.ny || h.nz != want.nz ||
      h.precision != want.precision || h.hydro_q != want.hydro_q || h.cac_solver != want.cac_solver ||
      h.hydro_store != want.hydro_store)
    return c->fail(LBM_E_INVALID, "state does not match this context (box, precision, lattice or solver)");
  HIP_OR_FAIL(c, hipStreamSynchronize(c->stream));
  HIP_OR_FAIL(c, hipMemcpy(c->ws, (const char*)buf + sizeof(h), pop_bytes(c), hipMemcpyHostToDevice));
  c->phi_cur = 0;
  if (c->fd())
    HIP_OR_FAIL(c, hipMemcpy(c->phi(), (const char*)buf + sizeof(h) + pop_bytes(c), phi_state_bytes(c),
                             hipMemcpyHostToDevice));
  c->step = h.step;
  c->mom_cur = (int)h.store_cur;
  c->dispersed = (int)h.dispersed;
  c->phys.rho_mean = h.rho_mean;
  reset_nci_state(c);
  HIP_OR_FAIL(c, hipStreamSynchronize(c->stream));
  c->hist_count = 0;
  c->initialised = true;
  return LBM_OK;
}

int lbm_nci_select(lbm_ctx* c, int mode) {
  if (!c) return LBM_E_INVALID;
  if (mode < -1 || mode > 1) return c->fail(LBM_E_INVALID, "nci_select mode must be -1, 0 or 1");
  HIP_OR_FAIL(c, hipStreamSynchronize(c->stream));
  c->nci_select = mode;
  return LBM_OK;
}

int lbm_force_wide_offsets(lbm_ctx* c, int on) {
  if (!c) return LBM_E_INVALID;
  HIP_OR_FAIL(c, hipStreamSynchronize(c->stream));
  c->wide_offsets = on != 0;
  return LBM_OK;
}

int lbm_timing(lbm_ctx* c, int enable) {
  if (!c) return LBM_E_INVALID;
  if (enable && c->ev.empty()) {
    c->ev.resize(2 * EV_PAIRS);
    c->ev_kind.resize(EV_PAIRS);
    for (auto& e : c->ev) HIP_OR_FAIL(c, hipEventCreate(&e));
  }
  if (!enable) {
    const int rc = flush_timing(c);
    if (rc != LBM_OK) return rc;
  }
  c->timing = enable != 0;
  return LBM_OK;
}

int lbm_kernel_times(lbm_ctx* c, double* ms, long* counts) {
  if (!c || !ms || !counts) return LBM_E_INVALID;
  const int rc = flush_timing(c);
  if (rc != LBM_OK) return rc;
  for (int k = 0; k < 5; ++k) {
    ms[k] = c->k_ms[k];
    counts[k] = c->k_cnt[k];
    c->k_ms[k] = 0.0;
    c->k_cnt[k] = 0;
  }
  return LBM_OK;
}

}  // extern "C"

namespace {
// Checks shared by the batch entry points; LBM_OK when the list may be stepped.
int check_batch(lbm_ctx* const* ctxs, int count) {
  lbm_ctx* c0 = ctxs[0];
  for (int i = 0; i < count; ++i) {
    lbm_ctx* c = ctxs[i];
    if (!c) return c0->fail(LBM_E_INVALID, "null context in batch");
    if (!c->initialised) return c0->fail(LBM_E_STATE, "batch holds an uninitialised context");
    if (c->fd())
      return c0->fail(LBM_E_UNSUPPORTED, "batches step the lattice Boltzmann phase field only (cac_solver 0)");
    if (c->mom())
      return c0->fail(LBM_E_UNSUPPORTED, "batches step the AA population storage only (hydro_store 0)");
    if (c->dev != c0->dev || c->p.dim != c0->p.dim || c->p.precision != c0->p.precision ||
        q_hydro(&c->p) != q_hydro(&c0->p))
      return c0->fail(LBM_E_INVALID, "batch contexts must share device, lattice and precision");
    for (int j = 0; j < i; ++j)
      if (ctxs[j] == c) return c0->fail(LBM_E_INVALID, "context listed twice in batch");
  }
  return LBM_OK;
}
}  // namespace

extern "C" {

int lbm_batch_step(lbm_ctx* const* ctxs, int count, int n) {
  if (!ctxs || count < 0 || n < 0) return LBM_E_INVALID;
  if (count == 0 || n == 0) return LBM_OK;
  lbm_ctx* c0 = ctxs[0];
  if (!c0) return LBM_E_INVALID;
  const int rc = check_batch(ctxs, count);
  if (rc != LBM_OK) return rc;
  return dispatch(c0, [&](auto E) { return decltype(E)::batch(ctxs, count, n); });
}

int lbm_batch_step_noalloc(lbm_ctx* const* ctxs, int count, int n) {
  if (!ctxs || count < 0 || n < 0) return LBM_E_INVALID;
  if (count == 0 || n == 0) return LBM_OK;
  lbm_ctx* c0 = ctxs[0];
  if (!c0) return LBM_E_INVALID;
  if (count > STATIC_JOBS)
    return c0->fail(LBM_E_INVALID, "lbm_batch_step_noalloc advances at most " + std::to_string(STATIC_JOBS) +
                                       " contexts per call (its job table is a fixed device array)");
  int rc = check_batch(ctxs, count);
  if (rc != LBM_OK) return rc;
  void* table = nullptr;
  std::string why;
  rc = scratch_on(c0->dev, &table, &why);
  if (rc != LBM_OK) return c0->fail(rc, why);
  return dispatch(c0, [&](auto E) {
    using En = decltype(E);
    return En::batch_noalloc(ctxs, count, n, (typename En::JobT*)table);
  });
}

}  // extern "C"
