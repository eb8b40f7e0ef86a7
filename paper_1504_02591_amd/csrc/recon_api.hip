// Host orchestration and C ABI of the reconstruction library.
//
// One plan owns a caller-provided device workspace carved into the buffers of
// the pipeline; all kernels run on the plan's stream.  The iteration keeps
// three complex work arrays (W0..W2) that cycle through
//   state X (x-inverse output of P_n)  --y_fanout-->  state Y (displacement spectra
//   inverse-transformed along y)  --z_iter, y_fanin, x_iter-->  state X,
// plus D_s and D_n.  Convergence norms come back as one small device-to-host
// copy per pass.
#include <hip/hip_runtime.h>
#include <rocprofiler-sdk-roctx/roctx.h>

#include <cmath>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "../../include/recon.h"
#include "../../include/recon_cnn.h"
#include "recon_cnn.hpp"
#include "recon_kernels.hpp"

using namespace recon;

namespace {

constexpr size_t kAlign = 256;
size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

enum PlanState { ST_EMPTY = 0, ST_PAINTED = 1, ST_DELTA = 2, ST_SOLVED = 3 };

// State Y of a realisation (its displacement spectra inverse-transformed along x and y): absent,
// full (W0..W2 = Psi_x, Psi_y, Psi_z: what the output needs) or combined (W0 = r_x Psi_x + r_y Psi_y,
// W2 = Psi_z: what the z iteration needs).  Both fan-outs consume state X.
enum StateY { SY_NONE = 0, SY_FULL = 1, SY_COMB = 2 };

struct Layout {
  size_t grid_g = 0, grid_r = 0, mask = 0, w0 = 0, w1 = 0, w2 = 0, ds = 0, dn = 0, psi = 0, delta = 0,
         corr = 0, tw = 0, partials = 0, red = 0, totals = 0, thr = 0, dscal = 0, act = 0, err = 0, total = 0,
         sorted = 0, bcount = 0, bstart = 0, bcursor = 0, bsum = 0, bvalid = 0, slot = 0, stmp = 0, bhist = 0, status = 0,
         tpart = 0, zflag = 0, mflag = 0;
  // network buffers
  size_t a1 = 0, a2 = 0, d1 = 0, d2 = 0, ybuf = 0, dybuf = 0, upbuf = 0, wk2t = 0, w3 = 0,
         part_out = 0, part_w1 = 0, part_w2 = 0, g1 = 0, g2 = 0, g3 = 0, grad = 0, lossp = 0, losst = 0, dc = 0, uc = 0,
         wf1 = 0, wf2 = 0, dh = 0, uh = 0;
  long long nb_conv = 0, nb_w = 0, nb_loss = 0;
  long long cnn_n = 0;
  long long nbins = 0, nscan = 0;
};

// Coarsening levels of the network grid: 0 (solver grid), 1 (RECON_CNN_HALF), 2 (RECON_CNN_QUARTER).
int cnn_levels(uint32_t flags) { return (flags & RECON_CNN_QUARTER) ? 2 : ((flags & RECON_CNN_HALF) ? 1 : 0); }

bool valid_params(const recon_params_t* p, std::string* why) {
  auto fail = [&](const char* m) { if (why) *why = m; return false; };
  if (!p) return fail("params is NULL");
  if (p->n < 8 || p->n > 1024 || (p->n & (p->n - 1))) return fail("n must be a power of two in [8, 1024]");
  if (p->batch < 1) return fail("batch must be >= 1");
  if (!(p->box_len > 0.0) || !std::isfinite(p->box_len)) return fail("box_len must be positive and finite");
  for (int a = 0; a < 3; ++a)
    if (!std::isfinite(p->box_origin[a]) || !std::isfinite(p->observer[a])) return fail("origin/observer must be finite");
  if (!(p->bias > 0.0) || !std::isfinite(p->bias)) return fail("bias must be positive and finite");
  if (!(p->growth >= 0.0) || !std::isfinite(p->growth)) return fail("growth must be >= 0 and finite");
  if (!(p->smooth_r >= 0.0) || !std::isfinite(p->smooth_r)) return fail("smooth_r must be >= 0 and finite");
  if (!(p->mask_tau >= 0.0) || !std::isfinite(p->mask_tau)) return fail("mask_tau must be >= 0 and finite");
  if (p->flags & ~(RECON_NO_RANDOMS | RECON_KEEP_DELTA | RECON_START_BUFFERS | RECON_CNN_BUFFERS | RECON_CNN_HALF |
                   RECON_PASS_GRAPHS | RECON_LOGNORMAL | RECON_FFT_SPLITBF16 | RECON_FFT_SPLITBF16_X3 |
                   RECON_CNN_QUARTER | RECON_RELAXED))
    return fail("unknown flag");
  if ((p->flags & RECON_FFT_SPLITBF16) && (p->flags & RECON_FFT_SPLITBF16_X3))
    return fail("RECON_FFT_SPLITBF16 and RECON_FFT_SPLITBF16_X3 exclude each other");
  if ((p->flags & (RECON_CNN_HALF | RECON_CNN_QUARTER)) && !(p->flags & RECON_CNN_BUFFERS))
    return fail("RECON_CNN_HALF / RECON_CNN_QUARTER need RECON_CNN_BUFFERS");
  if ((p->flags & RECON_CNN_HALF) && (p->flags & RECON_CNN_QUARTER))
    return fail("RECON_CNN_HALF and RECON_CNN_QUARTER exclude each other");
  if ((p->flags & RECON_CNN_BUFFERS) && (p->n >> cnn_levels(p->flags)) < 16)
    return fail("the network grid needs at least 16^3 cells");
  if (p->max_objects < 0 || p->max_objects >= (1LL << 32)) return fail("max_objects must be in [0, 2^32)");
  return true;
}

long long max_partial_blocks(int n) {
  // blocks of the reducing launches: x passes hold tile_x rows (per size), z passes >= 2 columns
  const int tx = n == 256 ? RECON_TILE_X_256 : (n == 1024 ? RECON_TILE_X_1024 : RECON_TILE_X);
  long long xb = (long long)(n / 2 + 1) * n / tx;
  long long zb = (long long)n * n / 2;
  return xb > zb ? xb : zb;
}

Layout make_layout(const recon_params_t* p) {
  Layout L;
  const long long n = p->n, b = p->batch;
  const long long n3 = n * n * n, cn = (n / 2 + 1) * n * n;
  const bool randoms = !(p->flags & RECON_NO_RANDOMS);
  size_t off = 0;
  auto take = [&](size_t bytes) { size_t o = off; off = align_up(off + bytes); return o; };
  L.grid_g = take(b * n3 * 8);
  L.grid_r = randoms ? take(b * n3 * 8) : 0;
  L.mask = randoms ? take(b * n3) : 0;
  L.w0 = take(b * cn * 8);
  L.w1 = take(b * cn * 8);
  L.w2 = take(b * cn * 8);
  L.ds = take(b * cn * 8);
  L.dn = take(b * cn * 8);
  L.psi = take(b * n3 * 12);
  L.delta = (p->flags & RECON_KEEP_DELTA) ? take(b * n3 * 4) : 0;
  L.corr = (p->flags & RECON_START_BUFFERS) ? take(b * n3 * 4) : 0;
  L.tw = take(n * 8);
  L.partials = take((size_t)b * max_partial_blocks((int)n) * 2 * 8);
  L.red = take(b * 2 * 8 * 2);
  L.totals = take(b * 3 * 8);
  L.thr = take(b * 8);
  L.status = take(b * 4);
  L.tpart = take((size_t)b * max_partial_blocks((int)n) * 3 * 8);
  L.dscal = take(b * sizeof(DeltaScal));
  L.act = take(b * 4 * 4);
  L.err = take(16);
  // tile flags of the setup transforms (one byte per z tile; n^2 bytes bound the tile count)
  L.zflag = take((size_t)(randoms ? 2 : 1) * b * n * n);
  L.mflag = randoms ? take((size_t)b * n * n) : 0;
  if (p->max_objects > 0) {
    const long long nbs = (n + kBrick - 1) / kBrick;
    L.nbins = b * nbs * nbs * nbs;
    L.nscan = (L.nbins + 256LL * kScanItems - 1) / (256LL * kScanItems);
    L.sorted = take((size_t)p->max_objects * 16);
    L.slot = take((size_t)p->max_objects * 4);
    L.stmp = take((size_t)p->max_objects * 16);
    L.bcount = take((L.nbins + 2) * 4);
    L.bstart = take((L.nbins + 2) * 4);
    L.bcursor = take((L.nbins + 2) * 4);
    L.bsum = take(L.nscan * 4);
    L.bhist = take((size_t)RECON_BIN_BLOCKS * kLdsBins * 4);
    L.bvalid = take(2 * L.nbins);
  }
  if (p->flags & RECON_CNN_BUFFERS) {
    using namespace recon::cnn;
    const int lv = cnn_levels(p->flags);
    const long long m = n >> lv, m3 = m * m * m;   // network grid
    L.cnn_n = m;
    L.nb_conv = m3 / TPOS;
    L.nb_w = (m / TY) * (m / TZ);
    L.nb_loss = 1024;
    L.a1 = take(b * m3 * CH * 2);
    L.a2 = take(b * m3 * CH * 2);
    L.d1 = take(b * m3 * CH * 2);
    L.d2 = take(b * m3 * CH * 2);
    L.ybuf = take(b * m3 * 4);
    L.dybuf = take(b * m3 * 4);
    L.upbuf = take(b * n3 * 4);
    if (lv >= 1) {
      // restricted inputs on the network grid; with two levels also the (n/2)^3 intermediates
      // (the second also holds the network output prolonged once)
      L.dc = take(b * m3 * 4);
      L.uc = take(b * m3 * 4);
    }
    if (lv == 2) {
      // (n/2)^3 intermediates of the two-step restriction
      const long long h3 = (n / 2) * (n / 2) * (n / 2);
      L.dh = take(b * h3 * 4);
      L.uh = take(b * h3 * 4);
    }
    L.wk2t = take(CH * K2 * 2);
    L.w3 = take(K2 * 4);
    L.wf1 = take(9 * 64 * 16);
    L.wf2 = take(9 * 2 * 64 * 16);
    L.part_out = take((size_t)b * L.nb_conv * (K2 + 1) * 4);
    L.part_w1 = take((size_t)b * L.nb_w * CH * (K1P + 1) * 4);
    L.part_w2 = take((size_t)b * L.nb_w * CH * (K2 + 1) * 4);
    L.g1 = take(CH * (K1P + 1) * 4);
    L.g2 = take(CH * (K2 + 1) * 4);
    L.g3 = take((K2 + 1) * 4);
    L.grad = take(NPARAM * 4);
    L.lossp = take(L.nb_loss * 8);
    L.losst = take(8);
  }
  L.total = off;
  return L;
}

// Per-kernel event timing on the plan's stream (instrumentation; off by default).
enum KernelId {
  KP_FILL, KP_PAINT, KP_TOTALS, KP_MASK, KP_Z_FWD_GRID, KP_Y_FWD, KP_X_SMOOTH, KP_Y_INV, KP_Z_DELTA, KP_X_START,
  KP_Z_FWD_REAL, KP_Y_FANOUT, KP_Z_ITER, KP_Y_FANIN, KP_X_ITER, KP_REDUCE, KP_Z_FINAL, KP_SHIFT, KP_BIN, KP_SCAN,
  KP_CNN_FWD, KP_CNN_BWD, KP_RESAMPLE, KP_COUNT
};
const char* const kKernelNames[KP_COUNT] = {
    "fill", "paint", "totals", "mask", "z_fwd_grid", "y_fwd", "x_smooth", "y_inv", "z_delta", "x_start",
    "z_fwd_real", "y_fanout", "z_iter", "y_fanin", "x_iter", "reduce", "z_final", "shift", "bin", "scan",
    "cnn_fwd", "cnn_bwd", "resample"};

struct Profiler {
  bool on = false;
  std::vector<hipEvent_t> pool;
  size_t used = 0;
  std::vector<std::pair<int, size_t>> recs;
};

}  // namespace

// Small host buffer for the per-pass read-backs of the convergence sums: pinned memory
// (hipHostMalloc), so that the copy is a direct DMA instead of a staged copy into pageable memory, or
// ordinary host memory for a plan that may not call HIP allocation routines.
struct PinnedDoubles {
  double* p = nullptr;
  size_t n = 0;
  bool pinned = true;
  PinnedDoubles() = default;
  PinnedDoubles(const PinnedDoubles&) = delete;
  PinnedDoubles& operator=(const PinnedDoubles&) = delete;
  ~PinnedDoubles() { release(); }
  void release() {
    if (p) {
      if (pinned) (void)hipHostFree(p);
      else delete[] p;
    }
    p = nullptr;
    n = 0;
  }
  bool assign(size_t count, double v, bool pin) {
    release();
    pinned = pin;
    if (pin) {
      if (hipHostMalloc((void**)&p, count * sizeof(double), hipHostMallocDefault) != hipSuccess) p = nullptr;
    } else {
      p = new (std::nothrow) double[count];
    }
    if (!p) return false;
    n = count;
    for (size_t i = 0; i < count; ++i) p[i] = v;
    return true;
  }
  double* data() { return p; }
  double& operator[](size_t i) { return p[i]; }
};

// The library's own device scratch for plans that cannot allocate (recon_plan_noalloc): one array per
// GPU, held until the process ends.  Host code never uses the symbol itself as an address (there it
// is only a host-side stand-in); the device address of each GPU's copy comes from
// hipGetSymbolAddress, taken once per device with that device current.
constexpr size_t kScratchBytes = 64ull << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
struct ScratchSlot {
  void* ptr = nullptr;             // device address of this GPU's scratch
  unsigned long long owner = 0;    // generation of the no-allocation plan that holds it (0: none)
  unsigned long long next = 0;
};
std::mutex g_scratch_mu;
ScratchSlot g_scratch[kMaxDevices];
}  // namespace

struct recon_plan_s {
  recon_params_t p{};
  // a plan on the library's scratch (recon_plan_noalloc): its device and generation; -1 otherwise
  int scratch_dev = -1;
  unsigned long long scratch_gen = 0;
  hipStream_t stream = nullptr;
  char* ws = nullptr;
  Layout L;
  int n = 0, batch = 1;
  long long n3 = 0, cn = 0;
  bool randoms = true;
  long long *grid_g = nullptr, *grid_r = nullptr;
  unsigned char* mask = nullptr;
  float2 *w0 = nullptr, *w1 = nullptr, *w2 = nullptr, *ds = nullptr, *dn = nullptr, *tw = nullptr;
  float* psi = nullptr;   // planar [batch][3][N^3]
  float *delta = nullptr, *corr = nullptr;
  double *partials = nullptr, *red = nullptr;
  unsigned long long* totals = nullptr;
  unsigned long long* tpart = nullptr;
  long long* thr = nullptr;
  int* status = nullptr;
  DeltaScal* dscal = nullptr;
  int *act_fan = nullptr, *act_fin = nullptr, *act_it = nullptr, *err = nullptr;
  float4* sorted = nullptr;
  // the brick-ordered copy of the catalogue painted last through the bricks: slot of every object
  // (input order), displacement staging for the shift in brick order, and which call it came from
  unsigned* slot_of = nullptr;
  float4* stmp = nullptr;
  int srt_which = -1;
  const float* srt_pos = nullptr;
  long long srt_n = 0;
  const int64_t* srt_off = nullptr;
  unsigned short *a1 = nullptr, *a2 = nullptr, *d1 = nullptr, *d2 = nullptr,
                 *wk2t = nullptr;
  float *ybuf = nullptr, *dybuf = nullptr, *upbuf = nullptr, *w3 = nullptr, *part_out = nullptr,
        *part_w1 = nullptr, *part_w2 = nullptr, *g1 = nullptr, *g2 = nullptr, *g3 = nullptr, *gradbuf = nullptr,
        *dc = nullptr, *uc = nullptr, *dh = nullptr, *uh = nullptr;
  uint4 *wf1 = nullptr, *wf2 = nullptr;
  int cnn_n = 0;                 // network grid: n, or n/2 with RECON_CNN_HALF
  long long cnn_n3 = 0;
  double *lossp = nullptr, *losst = nullptr;
  const float* net = nullptr;
  unsigned *bcount = nullptr, *bstart = nullptr, *bcursor = nullptr, *bsum = nullptr;
  unsigned* bhist = nullptr;   // per-block LDS histograms of the binning count, reused by the scatter
  // brick-sparse integer grids: per-brick validity of each grid, used while sparse_* is set (the
  // bricks that are not valid are zero and are not read)
  unsigned char *bvalid_g = nullptr, *bvalid_r = nullptr;
  // z-tile flags of the setup: grid tiles written by the forward z pass ([arrays][batch][tiles]) and
  // tiles with any cell inside the survey mask ([batch][tiles])
  unsigned char *zflag = nullptr, *mflag = nullptr;
  bool sparse_g = false, sparse_r = false;
  Geo geo{};
  CicGeo cic{};
  bool painted_g = false, painted_r = false;
  int state = ST_EMPTY;
  int start = RECON_START_PLAIN;
  // start of each realisation (a learned start that is rejected restarts from the plain start) and
  // how often that happened since the solve
  std::vector<int> start_b, restarts;
  std::vector<int> passes, done, psi_valid, st_y, pending1, diverged, stale_x;
  std::vector<double> num0, den0, s1, s2, norm1;
  std::vector<std::vector<double>> hist;
  std::vector<int> h_fan, h_fin, h_it;
  std::vector<int> up_fan, up_fin, up_it;     // what the device masks hold (empty: not yet uploaded)
  PinnedDoubles h_red, h_red2;
  std::string msg;
  Profiler prof;
  // steady-state pass graph (RECON_PASS_GRAPHS): fan-out, z step, fan-in, x step, norm reduction
  hipStream_t cap_stream = nullptr;
  hipGraphExec_t pass_graph = nullptr;
  ~recon_plan_s() {
    for (hipEvent_t e : prof.pool) (void)hipEventDestroy(e);
    if (pass_graph) (void)hipGraphExecDestroy(pass_graph);
    if (cap_stream) (void)hipStreamDestroy(cap_stream);
  }
};

namespace {

int fail(recon_plan_t* pl, int code, const std::string& m) {
  if (pl) pl->msg = m;
  return code;
}

int check_launch(recon_plan_t* pl, const char* what) {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(pl, RECON_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
  return RECON_OK;
}

// roctx range over a stage of the pipeline (host side: the enqueueing of its launches, and the waits
// of the calls that synchronise), named after the hot-path step it covers.
struct Marker {
  explicit Marker(const char* m) { roctxRangePushA(m); }
  ~Marker() { roctxRangePop(); }
  Marker(const Marker&) = delete;
  Marker& operator=(const Marker&) = delete;
};

struct ProfScope {
  recon_plan_t* pl;
  size_t idx = 0;
  bool live = false;
  ProfScope(recon_plan_t* p, int id) : pl(p) {
    Profiler& pr = pl->prof;
    if (!pr.on) return;
    while (pr.pool.size() < pr.used + 2) {
      hipEvent_t e;
      if (hipEventCreate(&e) != hipSuccess) return;
      pr.pool.push_back(e);
    }
    idx = pr.used;
    pr.used += 2;
    (void)hipEventRecord(pr.pool[idx], pl->stream);
    pr.recs.emplace_back(id, idx);
    live = true;
  }
  ~ProfScope() {
    if (live) (void)hipEventRecord(pl->prof.pool[idx + 1], pl->stream);
  }
};
#define PROF_CAT2(a, b) a##b
#define PROF_CAT(a, b) PROF_CAT2(a, b)
#define PROF(pl, id) ProfScope PROF_CAT(prof_scope_, __LINE__)(pl, id)

#define RECON_TRY(expr)          \
  do {                           \
    int rc_ = (expr);            \
    if (rc_ != RECON_OK) return rc_; \
  } while (0)

#define HIP_TRY(pl, call)                                                           \
  do {                                                                              \
    hipError_t e_ = (call);                                                         \
    if (e_ != hipSuccess) return fail(pl, RECON_EDEVICE, std::string(#call) + ": " + hipGetErrorString(e_)); \
  } while (0)

// ---------------------------------------------------------------------------
// Per-size launchers
// ---------------------------------------------------------------------------
struct Ops {
  int (*setup)(recon_plan_t*);             // z/y/x/y/z/y/x chain from the painted grids to D_s and state X
  int (*setup_delta)(recon_plan_t*, const float*);
  int (*fanout)(recon_plan_t*, const int*, bool comb);   // comb: combined state Y for the z iteration
  int (*combine)(recon_plan_t*, const int*);              // full state Y -> combined state Y
  int (*ziter)(recon_plan_t*, int mode, const int*);
  int (*fanin_xiter)(recon_plan_t*, bool first, const int*, float omega);
  int (*zfinal)(recon_plan_t*, float* psi, float* u, bool cross, const int*, bool comb);
  int (*refan)(recon_plan_t*, const int*, const float2* d);  // state X again from the spectrum d
  int (*helm)(recon_plan_t*, const float*);  // fan-out of the Helmholtz projection of a real field
  int nb_x, nb_z;
};

// Brick validity of a grid for its readers: null while the grid is dense.
const unsigned char* valid_of(const recon_plan_t* pl, int which) {
  if (which == RECON_GAL) return pl->sparse_g ? pl->bvalid_g : nullptr;
  return pl->sparse_r ? pl->bvalid_r : nullptr;
}

// Device-side alpha / rho_bar / mask threshold from the totals, then the survey mask.
int launch_fill_u64(recon_plan_t* pl, void* p, long long count);

// Scalars, and with randoms the survey mask and its z-tile flags (pl->mflag; tile width tw = 2 wz).
int scalars_and_mask(recon_plan_t* pl, int nblk_z, int tw) {
  k_scalars<<<pl->batch, 256, 0, pl->stream>>>(pl->tpart, nblk_z, pl->n3, pl->p.mask_tau, pl->randoms ? 1 : 0,
                                               pl->totals, pl->dscal, pl->thr, pl->status);
  RECON_TRY(check_launch(pl, "scalars"));
  if (pl->randoms) {
    const unsigned char* v = valid_of(pl, RECON_RAN);
    if (v && tw % kBrick == 0) {
      // the brick mask sets the flags of the tiles it writes into
      RECON_TRY(launch_fill_u64(pl, pl->mflag, ((long long)pl->batch * nblk_z + 7) / 8));
      PROF(pl, KP_MASK);
      k_mask_brick<<<(unsigned)pl->L.nbins, 256, 0, pl->stream>>>(pl->grid_r, pl->n, pl->thr, v, pl->mask, pl->mflag,
                                                                 tw);
    } else {
      {
        PROF(pl, KP_MASK);
        if (v) {
          k_mask_brick<<<(unsigned)pl->L.nbins, 256, 0, pl->stream>>>(pl->grid_r, pl->n, pl->thr, v, pl->mask);
        } else {
          const int nseg = (pl->n + 61) / 62;
          const unsigned blocks = (unsigned)(nseg * ((pl->n + 3) / 4));
          k_mask_win<<<dim3(blocks, pl->batch), 256, 0, pl->stream>>>(pl->grid_r, pl->n, pl->thr, pl->mask);
        }
      }
      RECON_TRY(check_launch(pl, "mask"));
      PROF(pl, KP_MASK);
      k_mask_tiles<<<dim3((unsigned)nblk_z, pl->batch), 256, 0, pl->stream>>>(pl->mask, pl->n, tw, pl->mflag);
    }
    RECON_TRY(check_launch(pl, "mask"));
  }
  return RECON_OK;
}

// Weight of the relaxed pass (RECON_RELAXED): 2/(2 + beta); 1 (the plain pass) without the flag.
float relax_weight(const recon_plan_t* pl) {
  if (!(pl->p.flags & RECON_RELAXED)) return 1.f;
  return (float)(2.0 / (2.0 + pl->p.growth / pl->p.bias));
}

// Lognormal option (RECON_LOGNORMAL): clamp of 1 + delta_s before the logarithm, 0 when off.
float log_floor(const recon_plan_t* pl) { return (pl->p.flags & RECON_LOGNORMAL) ? 1e-3f : 0.f; }

// C = -<ln(max(1 + delta_s, floor))> added to the kept field (the spectrum needs no change: C only
// moves the k = 0 mode, which does not enter Psi).
int log_constant(recon_plan_t* pl, int blocks) {
  if (!(pl->p.flags & RECON_LOGNORMAL) || !pl->delta) return RECON_OK;
  {
    PROF(pl, KP_REDUCE);
    k_reduce_pairs<<<pl->batch, 1024, 0, pl->stream>>>(pl->partials, blocks, pl->red + 2 * pl->batch);
  }
  RECON_TRY(check_launch(pl, "reduce (log mean)"));
  long long nb = (pl->n3 * pl->batch + 255) / 256;
  if (nb > 65536) nb = 65536;
  k_log_shift<<<(unsigned)nb, 256, 0, pl->stream>>>(pl->delta, pl->n3, pl->batch, pl->red + 2 * pl->batch);
  return check_launch(pl, "log shift");
}

template <int N>
struct SizeOps {
  static constexpr int WZ = wz<N>(), WY = wy<N>(), WX = wx<N>();
  static constexpr int TZ = ntz<N>(), TY = nty<N>(), TX = ntx<N>();
  static dim3 gz(const recon_plan_t* pl) { return dim3(N * (N / (2 * WZ)), pl->batch); }
  template <int MODE, int SPLIT = 0>
  static dim3 gzi(const recon_plan_t* pl) { return dim3(ztiles<N>() / ztpb<N, MODE, SPLIT>(), pl->batch); }
  static dim3 gy(const recon_plan_t* pl) { return dim3((N / 2 + 1) * (N / WY), pl->batch); }
  static dim3 gx(const recon_plan_t* pl) { return dim3((N / 2 + 1) * N / WX, pl->batch); }

  static int setup(recon_plan_t* pl) {
    hipStream_t s = pl->stream;
    if (pl->randoms) {
      {
        PROF(pl, KP_Z_FWD_GRID);
        k_z_fwd_grid<N, 2><<<gz(pl), dim3(TZ), 0, s>>>(pl->grid_g, pl->grid_r, pl->w0, pl->w1, pl->tpart, pl->tw,
                                                       valid_of(pl, RECON_GAL), valid_of(pl, RECON_RAN), pl->zflag);
      }
      RECON_TRY(check_launch(pl, "z forward (grids)"));
      // the mask (from the random grid and the totals) and its tile flags come first, so that the
      // inverse y pass can skip the rows the overdensity step will not read
      RECON_TRY(scalars_and_mask(pl, (int)gz(pl).x, 2 * WZ));
      {
        PROF(pl, KP_Y_FWD);
        k_y_plain<N, 2, false><<<gy(pl), dim3(TY), 0, s>>>(pl->w0, pl->w1, pl->tw, pl->zflag);
      }
      RECON_TRY(check_launch(pl, "y forward"));
      {
        PROF(pl, KP_X_SMOOTH);
        k_x_smooth<N, 2><<<gx(pl), dim3(TX), 0, s>>>(pl->w0, pl->w1, pl->geo, pl->tw);
      }
      RECON_TRY(check_launch(pl, "x smooth"));
      {
        PROF(pl, KP_Y_INV);
        k_y_plain<N, 2, true><<<gy(pl), dim3(TY), 0, s>>>(pl->w0, pl->w1, pl->tw, pl->mflag);
      }
      RECON_TRY(check_launch(pl, "y inverse"));
      {
        PROF(pl, KP_Z_DELTA);
        k_z_delta<N, 2><<<gz(pl), dim3(TZ), 0, s>>>(pl->w0, pl->w1, pl->mask, pl->dscal, pl->delta,
                                                    log_floor(pl), pl->partials, pl->tw, pl->mflag);
      }
      RECON_TRY(check_launch(pl, "z delta"));
      RECON_TRY(log_constant(pl, (int)gz(pl).x));
      return finish_start(pl, pl->mflag);
    } else {
      {
        PROF(pl, KP_Z_FWD_GRID);
        k_z_fwd_grid<N, 1><<<gz(pl), dim3(TZ), 0, s>>>(pl->grid_g, nullptr, pl->w0, nullptr, pl->tpart, pl->tw,
                                                       valid_of(pl, RECON_GAL), nullptr, pl->zflag);
      }
      RECON_TRY(check_launch(pl, "z forward (grid)"));
      {
        PROF(pl, KP_Y_FWD);
        k_y_plain<N, 1, false><<<gy(pl), dim3(TY), 0, s>>>(pl->w0, nullptr, pl->tw, pl->zflag);
      }
      RECON_TRY(check_launch(pl, "y forward"));
      {
        PROF(pl, KP_X_SMOOTH);
        k_x_smooth<N, 1><<<gx(pl), dim3(TX), 0, s>>>(pl->w0, nullptr, pl->geo, pl->tw);
      }
      RECON_TRY(check_launch(pl, "x smooth"));
      {
        PROF(pl, KP_Y_INV);
        k_y_plain<N, 1, true><<<gy(pl), dim3(TY), 0, s>>>(pl->w0, nullptr, pl->tw);
      }
      RECON_TRY(check_launch(pl, "y inverse"));
      RECON_TRY(scalars_and_mask(pl, (int)gz(pl).x, 2 * WZ));
      {
        PROF(pl, KP_Z_DELTA);
        k_z_delta<N, 1><<<gz(pl), dim3(TZ), 0, s>>>(pl->w0, nullptr, nullptr, pl->dscal, pl->delta,
                                                    log_floor(pl), pl->partials, pl->tw);
      }
      RECON_TRY(check_launch(pl, "z delta"));
      RECON_TRY(log_constant(pl, (int)gz(pl).x));
    }
    return finish_start(pl, nullptr);
  }

  // y and x forward of the overdensity's z spectrum (rows of the z tiles flagged 0 in mflag, when
  // given, were not written and are zero), D_s, and the fan-out state X of the plain start
  static int finish_start(recon_plan_t* pl, const unsigned char* mflag) {
    hipStream_t s = pl->stream;
    {
      PROF(pl, KP_Y_FWD);
      k_y_plain<N, 1, false><<<gy(pl), dim3(TY), 0, s>>>(pl->w0, nullptr, pl->tw, mflag);
    }
    RECON_TRY(check_launch(pl, "y forward (delta)"));
    {
      PROF(pl, KP_X_START);
      k_x_start<N><<<gx(pl), dim3(TX), 0, s>>>(pl->w0, pl->w1, pl->ds, pl->geo, pl->tw);
    }
    return check_launch(pl, "x start");
  }

  static int setup_delta(recon_plan_t* pl, const float* d) {
    {
      PROF(pl, KP_Z_FWD_REAL);
      k_z_fwd_real<N><<<gz(pl), dim3(TZ), 0, pl->stream>>>(d, pl->w0, pl->tw);
    }
    RECON_TRY(check_launch(pl, "z forward (delta)"));
    return finish_start(pl, nullptr);
  }

  // z and y forward of the field, then the HELM x start: the plan's fan-out state becomes that of
  // the irrotational projection (with the opposite sign)
  static int helm(recon_plan_t* pl, const float* f) {
    hipStream_t s = pl->stream;
    k_z_fwd_real<N><<<gz(pl), dim3(TZ), 0, s>>>(f, pl->w0, pl->tw);
    RECON_TRY(check_launch(pl, "z forward (Helmholtz)"));
    k_y_plain<N, 1, false><<<gy(pl), dim3(TY), 0, s>>>(pl->w0, nullptr, pl->tw);
    RECON_TRY(check_launch(pl, "y forward (Helmholtz)"));
    k_x_start<N, true><<<gx(pl), dim3(TX), 0, s>>>(pl->w0, pl->w1, pl->ds, pl->geo, pl->tw);
    return check_launch(pl, "x start (Helmholtz)");
  }

  static int refan(recon_plan_t* pl, const int* act, const float2* d) {
    {
      PROF(pl, KP_X_START);
      k_x_refan<N><<<gx(pl), dim3(TX), 0, pl->stream>>>(pl->w0, pl->w1, d, pl->geo, act, pl->tw);
    }
    return check_launch(pl, "x re-fan");
  }

  static int fanout(recon_plan_t* pl, const int* act, bool comb) {
    {
      PROF(pl, KP_Y_FANOUT);
      if (comb)
        k_y_fanout<N, true><<<gy(pl), dim3(TY), 0, pl->stream>>>(pl->w0, pl->w1, pl->w2, pl->geo, act, pl->tw);
      else
        k_y_fanout<N, false><<<gy(pl), dim3(TY), 0, pl->stream>>>(pl->w0, pl->w1, pl->w2, pl->geo, act, pl->tw);
    }
    return check_launch(pl, "y fan-out");
  }

  static int combine(recon_plan_t* pl, const int* act) {
    const long long cn = (long long)(N / 2 + 1) * N * N;
    long long nb = (cn + 255) / 256;
    if (nb > 8192) nb = 8192;
    k_y_combine<N><<<dim3((unsigned)nb, pl->batch), 256, 0, pl->stream>>>(pl->w0, pl->w1, pl->geo, act);
    return check_launch(pl, "y combine");
  }

  static int ziter(recon_plan_t* pl, int mode, const int* act) {
    hipStream_t s = pl->stream;
    {
      PROF(pl, KP_Z_ITER);
      if (mode == ZI_FFTA)
        k_z_iter<N, ZI_FFTA><<<gzi<ZI_FFTA>(pl), dim3(TZ), 0, s>>>(pl->w0, pl->w1, pl->w2, pl->geo, pl->corr,
                                                               pl->partials, act, pl->tw);
      else if (mode == ZI_LEARNED)
        k_z_iter<N, ZI_LEARNED><<<gzi<ZI_LEARNED>(pl), dim3(TZ), 0, s>>>(pl->w0, pl->w1, pl->w2, pl->geo, pl->corr,
                                                                  pl->partials, act, pl->tw, pl->upbuf);
      else if (mode == ZI_CROSS)
        k_z_iter<N, ZI_CROSS><<<gzi<ZI_CROSS>(pl), dim3(TZ), 0, s>>>(pl->w0, pl->w1, pl->w2, pl->geo, pl->corr,
                                                                pl->partials, act, pl->tw);
      else if (N >= 64 && (pl->p.flags & RECON_FFT_SPLITBF16))
        k_z_iter<N, ZI_PLAIN, N >= 64 ? 2 : 0><<<gzi<ZI_PLAIN, N >= 64 ? 2 : 0>(pl), dim3(TZ), 0, s>>>(
            pl->w0, pl->w1, pl->w2, pl->geo, nullptr, nullptr, act, pl->tw);
      else if (N >= 64 && (pl->p.flags & RECON_FFT_SPLITBF16_X3))
        k_z_iter<N, ZI_PLAIN, N >= 64 ? 3 : 0><<<gzi<ZI_PLAIN, N >= 64 ? 3 : 0>(pl), dim3(TZ), 0, s>>>(
            pl->w0, pl->w1, pl->w2, pl->geo, nullptr, nullptr, act, pl->tw);
      else if constexpr (N == 512 && RECON_Z_WAVE && wz<N>() == 16)
        k_z_iter_w<N><<<gzi<ZI_PLAIN>(pl), dim3(1024), 0, s>>>(pl->w0, pl->w1, pl->w2, pl->geo, act, pl->tw);
      else
        k_z_iter<N, ZI_PLAIN><<<gzi<ZI_PLAIN>(pl), dim3(TZ), 0, s>>>(pl->w0, pl->w1, pl->w2, pl->geo, nullptr,
                                                                nullptr, act, pl->tw);
    }
    RECON_TRY(check_launch(pl, "z iteration"));
    if (mode != ZI_PLAIN) {
      {
        PROF(pl, KP_REDUCE);
        // every mode other than the plain one runs one tile per block: the same grid
        k_reduce_pairs<<<pl->batch, 1024, 0, s>>>(pl->partials, (int)gzi<ZI_FFTA>(pl).x, pl->red + 2 * pl->batch);
      }
      RECON_TRY(check_launch(pl, "reduce (start sums)"));
    }
    return RECON_OK;
  }

  static int fanin_xiter(recon_plan_t* pl, bool first, const int* act, float omega) {
    hipStream_t s = pl->stream;
    {
      PROF(pl, KP_Y_FANIN);
      k_y_fanin<N><<<gy(pl), dim3(TY), 0, s>>>(pl->w0, pl->w1, pl->geo, act, pl->tw);
    }
    RECON_TRY(check_launch(pl, "y fan-in"));
    {
      PROF(pl, KP_X_ITER);
      k_x_iter<N><<<gx(pl), dim3(TX), 0, s>>>(pl->w0, pl->w1, pl->ds, first ? pl->ds : pl->dn, pl->dn,
                                                     pl->geo, pl->partials, act, pl->tw, omega);
    }
    RECON_TRY(check_launch(pl, "x iteration"));
    {
      PROF(pl, KP_REDUCE);
      k_reduce_pairs<<<pl->batch, 1024, 0, s>>>(pl->partials, (int)gx(pl).x, pl->red);
    }
    return check_launch(pl, "reduce (norm)");
  }

  static int zfinal(recon_plan_t* pl, float* psi, float* u, bool cross, const int* act, bool comb) {
    hipStream_t s = pl->stream;
    if (comb && (psi || cross)) return fail(pl, RECON_EINVAL, "internal: the combined state gives u only");
    {
      PROF(pl, KP_Z_FINAL);
      if (comb)
        k_z_final<N, true><<<gz(pl), dim3(TZ), 0, s>>>(pl->w0, pl->w1, pl->w2, pl->geo, nullptr, u, nullptr,
                                                       pl->partials, act, pl->tw);
      else
        k_z_final<N, false><<<gz(pl), dim3(TZ), 0, s>>>(pl->w0, pl->w1, pl->w2, pl->geo, psi, u,
                                                        cross ? pl->corr : nullptr, pl->partials, act, pl->tw);
    }
    RECON_TRY(check_launch(pl, "z final"));
    if (cross) {
      {
        PROF(pl, KP_REDUCE);
        k_reduce_pairs<<<pl->batch, 1024, 0, s>>>(pl->partials, (int)gz(pl).x, pl->red + 2 * pl->batch);
      }
      RECON_TRY(check_launch(pl, "reduce (cross sum)"));
    }
    return RECON_OK;
  }

  static const Ops* table() {
    static const Ops ops = {setup, setup_delta, fanout, combine, ziter, fanin_xiter, zfinal, refan, helm,
                            (int)((N / 2 + 1) * N / WX), (int)(N * (N / (2 * WZ)))};
    return &ops;
  }
};

const Ops* ops_for(int n) {
  switch (n) {
    case 8: return SizeOps<8>::table();
    case 16: return SizeOps<16>::table();
    case 32: return SizeOps<32>::table();
    case 64: return SizeOps<64>::table();
    case 128: return SizeOps<128>::table();
    case 256: return SizeOps<256>::table();
    case 512: return SizeOps<512>::table();
    case 1024: return SizeOps<1024>::table();
    default: return nullptr;
  }
}

int launch_fill_u64(recon_plan_t* pl, void* p, long long count) {
  long long blocks = (count + kThreads - 1) / kThreads;
  if (blocks > 65536) blocks = 65536;
  if (blocks < 1) blocks = 1;
  {
    PROF(pl, KP_FILL);
    k_fill_u64<<<(unsigned)blocks, kThreads, 0, pl->stream>>>((unsigned long long*)p, count);
  }
  return check_launch(pl, "fill");
}

// The device masks are written only here, so an upload whose flags the device copy already holds
// (the usual case from one pass to the next) is skipped.
int upload_mask(recon_plan_t* pl, int* dev, std::vector<int>& host) {
  std::vector<int>& held = dev == pl->act_fan ? pl->up_fan : (dev == pl->act_fin ? pl->up_fin : pl->up_it);
  if (held == host) return RECON_OK;
  held.clear();
  HIP_TRY(pl, hipMemcpyAsync(dev, host.data(), sizeof(int) * host.size(), hipMemcpyHostToDevice, pl->stream));
  held = host;
  return RECON_OK;
}

// Node geometry of the fine grid (level 0) or of the network grid (every (n / cnn_n)-th node).
recon::cnn::Geo3 grid_geo(const recon_plan_t* pl, bool network) {
  recon::cnn::Geo3 g;
  const int step = network ? pl->n / pl->cnn_n : 1;
  g.n = pl->n / step;
  g.hs = pl->geo.hs * (float)step;
  for (int a = 0; a < 3; ++a) g.ds[a] = pl->geo.ds[a];
  return g;
}
recon::cnn::Geo3 cnn_geo(const recon_plan_t* pl) { return grid_geo(pl, true); }

// Restriction of one field (fb == nullptr) or of two fields in one pass, from nf^3 (the plan's grid
// unless given) to (nf/2)^3.
int restrict_impl(recon_plan_t* pl, const float* fa, float* ca, const float* fb = nullptr, float* cb = nullptr,
                  int nf = 0) {
  if (nf == 0) nf = pl->n;
  const long long m = nf / 2;
  PROF(pl, KP_RESAMPLE);
  if (m >= 64) {   // slab kernel: 64 x 4 x 16 coarse nodes per block
    const dim3 grid((unsigned)((m / 64) * (m / 4) * (m / 16)), pl->batch);
    if (fb) recon::cnn::k_restrict_slab<2><<<grid, 256, 0, pl->stream>>>(fa, fb, nf, ca, cb);
    else recon::cnn::k_restrict_slab<1><<<grid, 256, 0, pl->stream>>>(fa, fa, nf, ca, ca);
  } else {
    const dim3 grid((unsigned)((m * m * m + 255) / 256), pl->batch);
    if (fb) recon::cnn::k_restrict<2><<<grid, 256, 0, pl->stream>>>(fa, fb, nf, ca, cb);
    else recon::cnn::k_restrict<1><<<grid, 256, 0, pl->stream>>>(fa, fa, nf, ca, ca);
  }
  return check_launch(pl, "restriction");
}

// Prolongation from (nf/2)^3 to nf^3 (the plan's grid unless given).
int prolong_impl(recon_plan_t* pl, const float* coarse, float scale, float* fine, int nf = 0) {
  if (nf == 0) nf = pl->n;
  const long long m = nf / 2;
  PROF(pl, KP_RESAMPLE);
  recon::cnn::k_prolong<<<dim3((unsigned)((m * m * m + 255) / 256), pl->batch), 256, 0, pl->stream>>>(coarse, nf,
                                                                                                      scale, fine);
  return check_launch(pl, "prolongation");
}

// Prolongation twice in one pass ((n/4)^3 -> n^3).
int prolong4_impl(recon_plan_t* pl, const float* coarse, float scale, float* fine) {
  const long long m = pl->n / 4;
  PROF(pl, KP_RESAMPLE);
  recon::cnn::k_prolong4<<<dim3((unsigned)((m * m * m + 255) / 256), pl->batch), 256, 0, pl->stream>>>(
      coarse, pl->n, scale, fine);
  return check_launch(pl, "prolongation (two levels)");
}

// Network forward on the plan's batch; out = scale * y.
int cnn_forward_impl(recon_plan_t* pl, const float* params, const float* delta, const float* up, float* out,
                     float scale) {
  using namespace recon::cnn;
  const dim3 grid((unsigned)pl->L.nb_conv, pl->batch);
  const Geo3 g = cnn_geo(pl);
  PROF(pl, KP_CNN_FWD);
  k_prep_weights<<<32, 256, 0, pl->stream>>>(params, pl->wk2t, pl->w3);
  k_prep_frag<<<(27 * 64 + 255) / 256, 256, 0, pl->stream>>>(params, pl->wf1, pl->wf2);
  const dim3 gridf((unsigned)(pl->cnn_n3 / (FX * FY * FZ)), pl->batch);
  k_conv_fwd<CIN, 1><<<gridf, 256, 0, pl->stream>>>(nullptr, delta, up, g, pl->wf1, params + OFF_B1, pl->a1);
  k_conv_fwd<CH, 0><<<gridf, 256, 0, pl->stream>>>(pl->a1, nullptr, nullptr, g, pl->wf2, params + OFF_B2, pl->a2);
  k_conv_out_mfma<<<gridf, 256, 0, pl->stream>>>(pl->a2, g, params + OFF_W3, params + OFF_B3, scale, out);
  return check_launch(pl, "network forward");
}

// Steady-state correction pass as a HIP graph: captured once per plan on a private stream (the
// plan's buffers, masks and geometry are fixed, so the recorded launches stay valid), then
// replayed on the plan's stream.  The graph holds kernels only (no memset or copy nodes); the
// activity masks it reads are uploaded before each replay.
int pass_graph_launch(recon_plan_t* pl, const Ops* ops) {
  if (!pl->pass_graph) {
    if (!pl->cap_stream) HIP_TRY(pl, hipStreamCreateWithFlags(&pl->cap_stream, hipStreamNonBlocking));
    hipStream_t keep = pl->stream;
    pl->stream = pl->cap_stream;
    hipGraph_t graph = nullptr;
    int rc = RECON_OK;
    if (hipStreamBeginCapture(pl->cap_stream, hipStreamCaptureModeRelaxed) != hipSuccess) {
      pl->stream = keep;
      return fail(pl, RECON_EDEVICE, "graph capture could not start");
    }
    rc = ops->fanout(pl, pl->act_fan, true);
    if (rc == RECON_OK) rc = ops->ziter(pl, ZI_PLAIN, pl->act_it);
    if (rc == RECON_OK) rc = ops->fanin_xiter(pl, false, pl->act_it, relax_weight(pl));
    const hipError_t ec = hipStreamEndCapture(pl->cap_stream, &graph);
    pl->stream = keep;
    if (rc != RECON_OK) {
      if (graph) (void)hipGraphDestroy(graph);
      return rc;
    }
    if (ec != hipSuccess || !graph) return fail(pl, RECON_EDEVICE, "graph capture failed");
    const hipError_t ei = hipGraphInstantiate(&pl->pass_graph, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (ei != hipSuccess) {
      pl->pass_graph = nullptr;
      return fail(pl, RECON_EDEVICE, "graph instantiation failed");
    }
  }
  HIP_TRY(pl, hipGraphLaunch(pl->pass_graph, pl->stream));
  return RECON_OK;
}

double ffta_c(int start, double beta) {
  if (start == RECON_START_FFTA1) return beta / (1.0 + beta);
  if (start == RECON_START_FFTA2) return 3.0 * beta / (7.0 + 3.0 * beta);
  return 0.0;
}

}  // namespace

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
extern "C" {

size_t recon_workspace_bytes(const recon_params_t* params) {
  if (!valid_params(params, nullptr)) return 0;
  return make_layout(params).total;
}

const char* recon_strerror(int code) {
  switch (code) {
    case RECON_OK: return "ok";
    case RECON_NOTCONVERGED: return "not converged within max_iter";
    case RECON_EINVAL: return "invalid argument";
    case RECON_ENOMEM: return "workspace too small";
    case RECON_EDEVICE: return "device error";
    case RECON_ESTATE: return "call out of order";
    case RECON_EDIVERGED: return "iteration diverged";
    default: return "unknown error";
  }
}

const char* recon_last_error(const recon_plan_t* plan) { return plan ? plan->msg.c_str() : "plan is NULL"; }

}  // extern "C"

namespace {

// A plan over `workspace` (validated by the callers); pinned: read-back buffers in pinned memory.
int plan_create(recon_plan_t** out, const recon_params_t* params, const Layout& L, void* workspace, void* stream,
                bool pinned) {
  recon_plan_t* pl = new (std::nothrow) recon_plan_t();
  if (!pl) return RECON_ENOMEM;
  pl->p = *params;
  pl->stream = (hipStream_t)stream;
  pl->ws = (char*)workspace;
  pl->L = L;
  pl->n = params->n;
  pl->batch = params->batch;
  pl->n3 = (long long)pl->n * pl->n * pl->n;
  pl->cn = (long long)(pl->n / 2 + 1) * pl->n * pl->n;
  pl->randoms = !(params->flags & RECON_NO_RANDOMS);
  char* w = pl->ws;
  pl->grid_g = (long long*)(w + L.grid_g);
  pl->grid_r = pl->randoms ? (long long*)(w + L.grid_r) : nullptr;
  pl->mask = pl->randoms ? (unsigned char*)(w + L.mask) : nullptr;
  pl->zflag = (unsigned char*)(w + L.zflag);
  pl->mflag = pl->randoms ? (unsigned char*)(w + L.mflag) : nullptr;
  pl->w0 = (float2*)(w + L.w0);
  pl->w1 = (float2*)(w + L.w1);
  pl->w2 = (float2*)(w + L.w2);
  pl->ds = (float2*)(w + L.ds);
  pl->dn = (float2*)(w + L.dn);
  pl->psi = (float*)(w + L.psi);
  pl->delta = (params->flags & RECON_KEEP_DELTA) ? (float*)(w + L.delta) : nullptr;
  pl->corr = (params->flags & RECON_START_BUFFERS) ? (float*)(w + L.corr) : nullptr;
  pl->tw = (float2*)(w + L.tw);
  pl->partials = (double*)(w + L.partials);
  pl->red = (double*)(w + L.red);
  pl->totals = (unsigned long long*)(w + L.totals);
  pl->thr = (long long*)(w + L.thr);
  pl->status = (int*)(w + L.status);
  pl->tpart = (unsigned long long*)(w + L.tpart);
  pl->dscal = (DeltaScal*)(w + L.dscal);
  pl->act_fan = (int*)(w + L.act);
  pl->act_fin = pl->act_fan + pl->batch;
  pl->act_it = pl->act_fan + 2 * pl->batch;
  pl->err = (int*)(w + L.err);
  if (params->flags & RECON_CNN_BUFFERS) {
    pl->a1 = (unsigned short*)(w + L.a1);
    pl->a2 = (unsigned short*)(w + L.a2);
    pl->d1 = (unsigned short*)(w + L.d1);
    pl->d2 = (unsigned short*)(w + L.d2);
    pl->ybuf = (float*)(w + L.ybuf);
    pl->dybuf = (float*)(w + L.dybuf);
    pl->upbuf = (float*)(w + L.upbuf);
    pl->wf1 = (uint4*)(w + L.wf1);
    pl->wf2 = (uint4*)(w + L.wf2);
    pl->cnn_n = (int)L.cnn_n;
    pl->cnn_n3 = L.cnn_n * L.cnn_n * L.cnn_n;
    if (params->flags & (RECON_CNN_HALF | RECON_CNN_QUARTER)) {
      pl->dc = (float*)(w + L.dc);
      pl->uc = (float*)(w + L.uc);
    }
    if ((params->flags & RECON_CNN_QUARTER) && L.dh) {
      pl->dh = (float*)(w + L.dh);
      pl->uh = (float*)(w + L.uh);
    }
    pl->wk2t = (unsigned short*)(w + L.wk2t);
    pl->w3 = (float*)(w + L.w3);
    pl->part_out = (float*)(w + L.part_out);
    pl->part_w1 = (float*)(w + L.part_w1);
    pl->part_w2 = (float*)(w + L.part_w2);
    pl->g1 = (float*)(w + L.g1);
    pl->g2 = (float*)(w + L.g2);
    pl->g3 = (float*)(w + L.g3);
    pl->gradbuf = (float*)(w + L.grad);
    pl->lossp = (double*)(w + L.lossp);
    pl->losst = (double*)(w + L.losst);
  }
  if (params->max_objects > 0) {
    pl->sorted = (float4*)(w + L.sorted);
    pl->slot_of = (unsigned*)(w + L.slot);
    pl->stmp = (float4*)(w + L.stmp);
    pl->bcount = (unsigned*)(w + L.bcount);
    pl->bstart = (unsigned*)(w + L.bstart);
    pl->bcursor = (unsigned*)(w + L.bcursor);
    pl->bsum = (unsigned*)(w + L.bsum);
    pl->bhist = (unsigned*)(w + L.bhist);
    pl->bvalid_g = (unsigned char*)(w + L.bvalid);
    pl->bvalid_r = pl->bvalid_g + L.nbins;
  }

  const int n = pl->n;
  const double L0 = params->box_len, h = L0 / n;
  // line-of-sight scale: a power of two >= every |origin - observer| and L, so scaling is exact
  double m = L0;
  for (int a = 0; a < 3; ++a) m = std::fmax(m, std::fabs(params->box_origin[a] - params->observer[a]));
  const double r0 = std::ldexp(1.0, (int)std::ceil(std::log2(m)));
  pl->geo.kf = (float)(2.0 * M_PI / L0);
  pl->geo.hs = (float)(h / r0);
  for (int a = 0; a < 3; ++a) pl->geo.ds[a] = (float)((params->box_origin[a] - params->observer[a]) / r0);
  pl->geo.growth = (float)params->growth;
  pl->geo.inv_bn3 = (float)(1.0 / (params->bias * (double)n * n * n));
  pl->geo.smooth_c = (float)(0.5 * params->smooth_r * params->smooth_r);
  pl->geo.inv_n3 = (float)(1.0 / ((double)n * n * n));
  pl->geo.start_scale = 1.0f;
  pl->cic.n = n;
  pl->cic.s = (float)((double)n / L0);
  for (int a = 0; a < 3; ++a) pl->cic.o[a] = (float)params->box_origin[a];
  pl->passes.assign(pl->batch, 0);
  pl->done.assign(pl->batch, 0);
  pl->psi_valid.assign(pl->batch, 0);
  pl->st_y.assign(pl->batch, 0);
  pl->pending1.assign(pl->batch, 0);
  pl->diverged.assign(pl->batch, 0);
  pl->stale_x.assign(pl->batch, 0);
  pl->start_b.assign(pl->batch, RECON_START_PLAIN);
  pl->restarts.assign(pl->batch, 0);
  pl->num0.assign(pl->batch, 0.0);
  pl->den0.assign(pl->batch, 0.0);
  pl->s1.assign(pl->batch, 0.0);
  pl->s2.assign(pl->batch, 0.0);
  pl->norm1.assign(pl->batch, 0.0);
  pl->hist.assign(pl->batch, {});
  pl->h_fan.assign(pl->batch, 0);
  pl->h_fin.assign(pl->batch, 0);
  pl->h_it.assign(pl->batch, 0);
  if (!pl->h_red.assign(4 * pl->batch, 0.0, pinned) || !pl->h_red2.assign(2 * pl->batch, 0.0, pinned)) {
    delete pl;
    return RECON_EDEVICE;
  }

  {
    const Ops* ops = ops_for(n);
    if (!ops || ops->nb_x > max_partial_blocks(n) || ops->nb_z > max_partial_blocks(n)) {
      delete pl;
      return RECON_EINVAL;
    }
  }
  // twiddles exp(-2 pi i m / N), rounded once from double
  std::vector<float2> tw(n);
  for (int i = 0; i < n; ++i) {
    const double ang = -2.0 * M_PI * (double)i / (double)n;
    tw[i] = make_float2((float)std::cos(ang), (float)std::sin(ang));
  }
  if (hipMemcpyAsync(pl->tw, tw.data(), sizeof(float2) * n, hipMemcpyHostToDevice, pl->stream) != hipSuccess ||
      hipStreamSynchronize(pl->stream) != hipSuccess) {
    delete pl;
    return RECON_EDEVICE;
  }
  *out = pl;
  return RECON_OK;
}

// A plan on the library's scratch is usable while no later recon_plan_noalloc took that scratch.
int check_scratch_owner(recon_plan_t* pl) {
  if (pl->scratch_dev < 0) return RECON_OK;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch[pl->scratch_dev].owner != pl->scratch_gen)
    return fail(pl, RECON_ESTATE, "a later recon_plan_noalloc on this device took the scratch this plan used");
  return RECON_OK;
}

}  // namespace

#define CHECK_PLAN(pl)                    \
  do {                                    \
    if (!(pl)) return RECON_EINVAL;       \
    RECON_TRY(check_scratch_owner(pl));   \
  } while (0)

extern "C" {

int recon_plan(recon_plan_t** out, const recon_params_t* params, void* workspace, size_t workspace_bytes,
               void* stream) {
  if (!out) return RECON_EINVAL;
  *out = nullptr;
  std::string why;
  if (!valid_params(params, &why)) return RECON_EINVAL;
  if (!workspace || ((uintptr_t)workspace % kAlign)) return RECON_EINVAL;
  Layout L = make_layout(params);
  if (workspace_bytes < L.total) return RECON_ENOMEM;
  return plan_create(out, params, L, workspace, stream, true);
}

size_t recon_noalloc_limit(void) { return kScratchBytes; }

int recon_plan_noalloc(recon_plan_t** out, const recon_params_t* params, void* stream) {
  if (!out) return RECON_EINVAL;
  *out = nullptr;
  std::string why;
  if (!valid_params(params, &why)) return RECON_EINVAL;
  if (params->flags & RECON_PASS_GRAPHS) return RECON_EINVAL;   // graph instantiation may allocate
  const Layout L = make_layout(params);
  if (L.total > kScratchBytes) return RECON_ENOMEM;
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return RECON_EDEVICE;
  void* ws = nullptr;
  unsigned long long gen = 0;
  {
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    ScratchSlot& slot = g_scratch[dev];
    if (!slot.ptr) {
      // once per device, with that device current: the device address of its copy of the array
      void* p = nullptr;
      if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return RECON_EDEVICE;
      slot.ptr = p;
    }
    ws = slot.ptr;
    gen = ++slot.next;
    slot.owner = gen;     // earlier no-allocation plans on this device are now stale
  }
  const int rc = plan_create(out, params, L, ws, stream, false);
  if (rc != RECON_OK) return rc;
  (*out)->scratch_dev = dev;
  (*out)->scratch_gen = gen;
  return RECON_OK;
}

void recon_destroy(recon_plan_t* plan) {
  if (plan && plan->scratch_dev >= 0) {
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (g_scratch[plan->scratch_dev].owner == plan->scratch_gen) g_scratch[plan->scratch_dev].owner = 0;
  }
  delete plan;
}

int recon_paint(recon_plan_t* pl, int which, const float* pos, const float* w, int64_t n, const int64_t* offsets,
                uint32_t flags) {
  CHECK_PLAN(pl);
  if (which != RECON_GAL && which != RECON_RAN) return fail(pl, RECON_EINVAL, "which must be RECON_GAL or RECON_RAN");
  if (which == RECON_RAN && !pl->randoms) return fail(pl, RECON_EINVAL, "plan was created with RECON_NO_RANDOMS");
  if (n < 0 || (n > 0 && !pos)) return fail(pl, RECON_EINVAL, "bad catalogue pointer or count");
  if (pl->batch > 1 && !offsets && n > 0) return fail(pl, RECON_EINVAL, "offsets are required when batch > 1");
  if (flags & ~(RECON_PAINT_ACCUMULATE | RECON_PAINT_NGP)) return fail(pl, RECON_EINVAL, "unknown paint flag");
  Marker mark(which == RECON_GAL ? "a1 deposit (galaxies)" : "a1 deposit (randoms)");
  long long* grid = which == RECON_GAL ? pl->grid_g : pl->grid_r;
  const bool first = which == RECON_GAL ? !pl->painted_g : !pl->painted_r;
  int* errc = pl->err + which;   // invalid-object counter of this grid
  const bool fresh = !(flags & RECON_PAINT_ACCUMULATE) || first;
  const bool binned = n > 0 && !(flags & RECON_PAINT_NGP) && n <= pl->p.max_objects;
  // brick-sparse grid: bricks tile the grid and the brick buffers exist
  const bool can_sparse = pl->L.nbins > 0 && pl->n >= 2 * kBrick;
  unsigned char* valid = which == RECON_GAL ? pl->bvalid_g : pl->bvalid_r;
  bool& sparse = which == RECON_GAL ? pl->sparse_g : pl->sparse_r;
  if (fresh) {
    HIP_TRY(pl, hipMemsetAsync(errc, 0, sizeof(int), pl->stream));
    if (!(binned && can_sparse)) {
      RECON_TRY(launch_fill_u64(pl, grid, pl->n3 * pl->batch));
      sparse = false;
    }   // else only the bricks the deposit touches are cleared, after the count below
  } else if (sparse && n > 0 && !binned) {
    // a deposit that does not go through the bricks adds into a dense grid: clear what is not valid
    {
      PROF(pl, KP_FILL);
      k_brick_prepare<<<(unsigned)pl->L.nbins, 256, 0, pl->stream>>>(pl->bcount, pl->n, 2, valid,
                                                                     (unsigned long long*)grid);
    }
    RECON_TRY(check_launch(pl, "brick densify"));
    sparse = false;
  }
  if (n > 0 && (flags & RECON_PAINT_NGP)) {
    long long blocks = (n + kThreads - 1) / kThreads;
    if (blocks > 8192) blocks = 8192;
    {
      PROF(pl, KP_PAINT);
      k_paint_ngp<<<(unsigned)blocks, kThreads, 0, pl->stream>>>(pos, w, n, (const long long*)offsets, pl->batch,
                                                                 (unsigned long long*)grid, pl->cic, errc);
    }
    RECON_TRY(check_launch(pl, "paint (NGP)"));
  } else if (binned) {
    // brick-binned deposit: count, scan, scatter into brick order, per-brick LDS accumulation
    pl->srt_which = -1;   // the sorted copy is being replaced
    long long blocks = (n + kThreads - 1) / kThreads;
    if (blocks > 8192) blocks = 8192;
    const long long nb = pl->L.nbins;
    RECON_TRY(launch_fill_u64(pl, pl->bcount, (nb + 2) / 2));
    const long long nbs = (pl->n + kBrick - 1) / kBrick;
    const bool lds_bins = RECON_BIN_WINDOW || nbs * nbs * nbs <= kLdsBins;   // windows above 512^3
    long long lblocks = (n + 16383) / 16384;
    if (lblocks > RECON_BIN_BLOCKS) lblocks = RECON_BIN_BLOCKS;
    const long long chunk = (n + lblocks - 1) / lblocks;
    {
      PROF(pl, KP_BIN);
      if (lds_bins)
        k_bin_count_lds<1024><<<(unsigned)lblocks, 1024, 0, pl->stream>>>(pos, w, n, chunk, (const long long*)offsets,
                                                                   pl->batch, pl->cic, pl->bcount, errc,
                                                                   pl->bhist);
      else
        k_bin_count<<<(unsigned)blocks, kThreads, 0, pl->stream>>>(pos, w, n, (const long long*)offsets, pl->batch,
                                                                   pl->cic, pl->bcount, errc);
    }
    RECON_TRY(check_launch(pl, "bin count"));
    if (can_sparse && (fresh || sparse)) {
      // clear the bricks this deposit touches (new grid), or those of them not held yet (accumulate)
      {
        PROF(pl, KP_FILL);
        k_brick_prepare<<<(unsigned)nb, 256, 0, pl->stream>>>(pl->bcount, pl->n, fresh ? 0 : 1, valid,
                                                              (unsigned long long*)grid);
      }
      RECON_TRY(check_launch(pl, "brick prepare"));
      sparse = true;
    }
    {
      PROF(pl, KP_SCAN);
      k_scan_blocks<<<(unsigned)pl->L.nscan, 256, 0, pl->stream>>>(pl->bcount, nb, pl->bsum);
      k_scan_top<<<1, 256, 0, pl->stream>>>(pl->bsum, (int)pl->L.nscan);
      k_scan_apply<<<(unsigned)pl->L.nscan, 256, 0, pl->stream>>>(pl->bcount, nb, pl->bsum, pl->bstart,
                                                                  pl->bcursor);
    }
    RECON_TRY(check_launch(pl, "bin scan"));
    {
      PROF(pl, KP_BIN);
      if (lds_bins)
        k_bin_scatter_lds<1024><<<(unsigned)lblocks, 1024, 0, pl->stream>>>(pos, w, n, chunk, (const long long*)offsets,
                                                                     pl->batch, pl->cic, pl->bcursor, pl->sorted,
                                                                     pl->slot_of, pl->bhist);
      else
        k_bin_scatter<<<(unsigned)blocks, kThreads, 0, pl->stream>>>(pos, w, n, (const long long*)offsets,
                                                                     pl->batch, pl->cic, pl->bcursor, pl->sorted,
                                                                     pl->slot_of);
    }
    RECON_TRY(check_launch(pl, "bin scatter"));
    {
      PROF(pl, KP_PAINT);
      k_brick_deposit<RECON_BRICK_NT><<<(unsigned)nb, RECON_BRICK_NT, 0, pl->stream>>>(pl->sorted, pl->bstart, pl->cic,
                                                            (unsigned long long*)grid);
    }
    RECON_TRY(check_launch(pl, "brick deposit"));
    pl->srt_which = which;
    pl->srt_pos = pos;
    pl->srt_n = n;
    pl->srt_off = offsets;
  } else if (n > 0) {
    long long blocks = (n + kThreads - 1) / kThreads;
    if (blocks > 8192) blocks = 8192;
    {
      PROF(pl, KP_PAINT);
      k_paint<<<(unsigned)blocks, kThreads, 0, pl->stream>>>(pos, w, n, (const long long*)offsets, pl->batch,
                                                             (unsigned long long*)grid, pl->cic, errc);
    }
    RECON_TRY(check_launch(pl, "paint"));
  }
  if (which == RECON_GAL) pl->painted_g = true; else pl->painted_r = true;
  pl->state = ST_PAINTED;
  return RECON_OK;
}

int recon_set_delta(recon_plan_t* pl, const float* delta_s) {
  CHECK_PLAN(pl);
  if (!delta_s) return fail(pl, RECON_EINVAL, "delta_s is NULL");
  const Ops* ops = ops_for(pl->n);
  if (pl->delta) {
    HIP_TRY(pl, hipMemcpyAsync(pl->delta, delta_s, sizeof(float) * pl->n3 * pl->batch, hipMemcpyDeviceToDevice,
                               pl->stream));
  }
  RECON_TRY(ops->setup_delta(pl, delta_s));
  pl->state = ST_DELTA;
  return RECON_OK;
}

int recon_solve(recon_plan_t* pl, int start, const void* net) {
  CHECK_PLAN(pl);
  if (start < RECON_START_PLAIN || start > RECON_START_LEARNED) return fail(pl, RECON_EINVAL, "unknown start");
  if (start != RECON_START_PLAIN && !pl->corr)
    return fail(pl, RECON_EINVAL, "non-plain starts need a plan created with RECON_START_BUFFERS");
  if (start == RECON_START_LEARNED) {
    if (!net) return fail(pl, RECON_EINVAL, "learned start needs the network parameters");
    if (!pl->delta || !pl->a1)
      return fail(pl, RECON_EINVAL, "learned start needs RECON_KEEP_DELTA and RECON_CNN_BUFFERS");
  }
  const Ops* ops = ops_for(pl->n);
  if (pl->state == ST_PAINTED) {
    if (!pl->painted_g) return fail(pl, RECON_ESTATE, "galaxies were not painted");
    if (pl->randoms && !pl->painted_r) return fail(pl, RECON_ESTATE, "randoms were not painted");
    Marker mark("a2-a6 totals, smoothing, mask, overdensity, D_s");
    RECON_TRY(ops->setup(pl));
    // one read-back: invalid-object counters and the totals status of every realisation
    std::vector<int> st(pl->batch, 0);
    int errs[2] = {0, 0};
    HIP_TRY(pl, hipMemcpyAsync(errs, pl->err, 2 * sizeof(int), hipMemcpyDeviceToHost, pl->stream));
    HIP_TRY(pl, hipMemcpyAsync(st.data(), pl->status, sizeof(int) * pl->batch, hipMemcpyDeviceToHost, pl->stream));
    HIP_TRY(pl, hipStreamSynchronize(pl->stream));
    const int errcount = errs[0] + (pl->randoms ? errs[1] : 0);
    if (errcount) return fail(pl, RECON_EINVAL, std::to_string(errcount) + " objects had invalid positions or weights");
    for (int b = 0; b < pl->batch; ++b) {
      if (st[b] & 1) return fail(pl, RECON_EINVAL, "total galaxy weight is zero");
      if (st[b] & 2) return fail(pl, RECON_EINVAL, "total random weight is zero");
    }

  } else if (pl->state != ST_DELTA && pl->state != ST_SOLVED) {
    return fail(pl, RECON_ESTATE, "paint or set_delta must precede solve");
  } else if (pl->state == ST_SOLVED) {
    return fail(pl, RECON_ESTATE, "already solved; paint or set_delta again");
  }
  pl->start = start;
  const double beta = pl->p.growth / pl->p.bias;
  pl->geo.start_scale = (float)(1.0 - ffta_c(start, beta));
  for (int b = 0; b < pl->batch; ++b) {
    pl->passes[b] = 0;
    pl->done[b] = 0;
    pl->psi_valid[b] = 0;
    pl->st_y[b] = SY_NONE;
    pl->pending1[b] = 0;
    pl->diverged[b] = 0;
    pl->stale_x[b] = 0;
    pl->hist[b].clear();
    pl->start_b[b] = start;
    pl->restarts[b] = 0;
  }
  if (start == RECON_START_LEARNED) {
    Marker mark("a7/a11 learned start (u_p, network)");
    // u_p = Psi_p . r_hat from the fanned-out start, then Delta u = network(delta_s, u_p) into corr
    RECON_TRY(ops->fanout(pl, nullptr, true));
    RECON_TRY(ops->zfinal(pl, nullptr, pl->upbuf, false, nullptr, true));
    if (pl->dh) {
      // network on the (n/4)^3 grid: two restrictions (both fields per pass), one trilinear
      // prolongation that equals the linear one applied twice
      RECON_TRY(restrict_impl(pl, pl->delta, pl->dh, pl->upbuf, pl->uh));
      RECON_TRY(restrict_impl(pl, pl->dh, pl->dc, pl->uh, pl->uc, pl->n / 2));
      RECON_TRY(cnn_forward_impl(pl, (const float*)net, pl->dc, pl->uc, pl->ybuf, 1.0f / recon::cnn::S_U));
      RECON_TRY(prolong4_impl(pl, pl->ybuf, 1.0f, pl->corr));
    } else if (pl->dc) {
      // network on the (n/2)^3 grid: restrict the inputs, prolong its output
      RECON_TRY(restrict_impl(pl, pl->delta, pl->dc, pl->upbuf, pl->uc));
      RECON_TRY(cnn_forward_impl(pl, (const float*)net, pl->dc, pl->uc, pl->ybuf, 1.0f / recon::cnn::S_U));
      RECON_TRY(prolong_impl(pl, pl->ybuf, 1.0f, pl->corr));
    } else {
      RECON_TRY(cnn_forward_impl(pl, (const float*)net, pl->delta, pl->upbuf, pl->corr, 1.0f / recon::cnn::S_U));
    }
    for (int b = 0; b < pl->batch; ++b) pl->st_y[b] = SY_COMB;
  }
  pl->state = ST_SOLVED;
  return RECON_OK;
}

// eps rising below this is rounding noise of a converged FP32 iteration, not divergence
constexpr double kEpsFloor = 1e-5;

// Upper bound of the plain start's eps_1 from the sums of a non-gradient start's first pass.  The
// map from a radial field u to Psi_1 - Psi_0 (Sec. 5.1, eq. iterative) is -beta k' (k' . FFT[u r])/k^2,
// whose norm is at most beta (|k'|^2 <= k^2, |r| <= 1).  With Psi_p the plain start, Psi_1 the
// learned start's first iterate and Delta the learned radial correction:
//   ||Psi_1 - Psi_1^plain|| <= beta ||Delta||,  ||Psi_1^plain - Psi_p|| <= beta ||Psi_p||,
// so eps_1^plain <= beta / (1 - beta) (beta < 1), and
//   eps_1^plain <= (||Psi_1 - Psi_p|| + beta ||Delta||) / (||Psi_1|| - beta ||Delta||).
// num0 = ||Psi_1 - Psi_p||^2, den0 = ||Psi_1||^2, s2 = ||Delta||^2 (configuration-space sums).
double plain_eps1_bound(double beta, double num0, double den0, double s2) {
  double bound = beta < 1.0 ? beta / (1.0 - beta) : INFINITY;
  const double bd = beta * std::sqrt(std::fmax(s2, 0.0)), dn = std::sqrt(std::fmax(den0, 0.0));
  if (dn > bd) bound = std::fmin(bound, (std::sqrt(std::fmax(num0, 0.0)) + bd) / (dn - bd));
  return bound;
}

int recon_iterate(recon_plan_t* pl, int max_iter, double tol, int32_t* iters_out, double* eps_out) {
  CHECK_PLAN(pl);
  if (pl->state != ST_SOLVED) return fail(pl, RECON_ESTATE, "solve must precede iterate");
  if (max_iter < 0) return fail(pl, RECON_EINVAL, "max_iter must be >= 0");
  const Ops* ops = ops_for(pl->n);
  const int B = pl->batch;
  const bool fixed = !(tol > 0.0);
  const double norm_k = 1.0 / (pl->p.bias * pl->p.bias * (double)pl->n3);   // Parseval + 1/b^2
  const double beta = pl->p.growth / pl->p.bias;
  std::vector<std::vector<double>> call_eps(B);
  for (int b = 0; b < B; ++b) pl->done[b] = pl->diverged[b] ? 1 : 0;
  bool restarted = false;

  // A rejected learned start: the realisation starts over from the plain start, D_0 = D_s.  Its D_n
  // becomes D_s (so that a pass reading D_n as the previous iterate starts from the plain start),
  // its state X is rebuilt from D_s before its next pass, and its history starts again.
  auto fall_back = [&](int b) -> int {
    HIP_TRY(pl, hipMemcpyAsync(pl->dn + (size_t)b * pl->cn, pl->ds + (size_t)b * pl->cn, sizeof(float2) * pl->cn,
                               hipMemcpyDeviceToDevice, pl->stream));
    pl->start_b[b] = RECON_START_PLAIN;
    pl->restarts[b] += 1;
    pl->passes[b] = 0;
    pl->pending1[b] = 0;
    pl->diverged[b] = 0;
    pl->done[b] = 0;
    pl->psi_valid[b] = 0;
    pl->st_y[b] = SY_NONE;
    pl->stale_x[b] = 1;
    pl->hist[b].clear();
    call_eps[b].clear();
    restarted = true;
    return RECON_OK;
  };

  // norm2 = ||Psi_n||^2.  Divergence: non-finite eps, eps rising twice in a row, or
  // ||Psi_n|| > 100 ||Psi_1||.  A learned start that diverges falls back to the plain start once.
  auto record = [&](int b, double e, double norm2) -> int {
    call_eps[b].push_back(e);
    pl->hist[b].push_back(e);
    const auto& h = pl->hist[b];
    const size_t k = h.size();
    // a non-finite norm (a non-finite field) must not be clipped to 0 and read as convergence
    const double nrm = std::isfinite(norm2) ? std::sqrt(std::fmax(norm2, 0.0)) : NAN;
    if (k == 1) pl->norm1[b] = nrm;
    if (!std::isfinite(e) || !std::isfinite(nrm) ||
        (k >= 3 && h[k - 1] > h[k - 2] && h[k - 2] > h[k - 3] && h[k - 1] > kEpsFloor) ||
        (k >= 2 && nrm > 100.0 * pl->norm1[b])) {
      if (pl->start_b[b] == RECON_START_LEARNED) return fall_back(b);
      pl->diverged[b] = 1;
      pl->done[b] = 1;
    } else if (!fixed && e <= tol) {
      pl->done[b] = 1;
    }
    return RECON_OK;
  };

  // eps_1 of a non-gradient start from the first pass's sums and S3 = sum Delta u_1.  A learned start
  // whose eps_1 is non-finite, or above the bound of the plain start's eps_1, is rejected: it is
  // provably a worse start than the plain one.  Returns whether the realisation fell back.
  auto judge_eps1 = [&](int b, double s3, bool& fell) -> int {
    fell = false;
    const double diff2 = pl->num0[b] - 2.0 * (s3 - pl->s1[b]) + pl->s2[b];
    const double e = !std::isfinite(diff2) ? NAN
                     : (pl->den0[b] > 0 ? std::sqrt(std::fmax(diff2, 0.0) / pl->den0[b]) : 0.0);
    if (pl->start_b[b] == RECON_START_LEARNED &&
        !(e <= plain_eps1_bound(beta, pl->num0[b], pl->den0[b], pl->s2[b]))) {
      fell = true;
      return fall_back(b);
    }
    return record(b, e, pl->den0[b]);
  };

  // state X again (from D_s before the first pass, else from D_n) for the realisations marked in
  // h_fan whose state X is gone
  auto rebuild_x = [&](const std::vector<int>& want) -> int {
    for (int pick = 0; pick < 2; ++pick) {
      bool any = false;
      for (int b = 0; b < B; ++b) {
        pl->h_fan[b] = (want[b] && (pl->passes[b] == 0) == (pick == 0)) ? 1 : 0;
        any = any || pl->h_fan[b];
      }
      if (!any) continue;
      RECON_TRY(upload_mask(pl, pl->act_fan, pl->h_fan));
      RECON_TRY(ops->refan(pl, pl->act_fan, pick == 0 ? pl->ds : pl->dn));
      for (int b = 0; b < B; ++b)
        if (pl->h_fan[b]) { pl->stale_x[b] = 0; pl->st_y[b] = SY_NONE; }
    }
    return RECON_OK;
  };

  // full state Y for the realisations marked in h_fin: state X is rebuilt first where it is gone
  // (a combined state Y, or a pass stopped after its z step) from D_n, or D_s before the first pass
  auto full_state = [&]() -> int {
    std::vector<int> want(B, 0);
    for (int b = 0; b < B; ++b) want[b] = pl->h_fin[b] && (pl->stale_x[b] || pl->st_y[b] == SY_COMB);
    RECON_TRY(rebuild_x(want));
    bool any = false;
    for (int b = 0; b < B; ++b) {
      pl->h_fan[b] = (pl->h_fin[b] && pl->st_y[b] != SY_FULL) ? 1 : 0;
      any = any || pl->h_fan[b];
    }
    if (any) {
      RECON_TRY(upload_mask(pl, pl->act_fan, pl->h_fan));
      RECON_TRY(ops->fanout(pl, pl->act_fan, false));
      for (int b = 0; b < B; ++b)
        if (pl->h_fan[b]) pl->st_y[b] = SY_FULL;
    }
    return RECON_OK;
  };

  // resolve eps_1 of a non-gradient start: needs the full state Y of D_1
  auto resolve_pending = [&]() -> int {
    bool any = false;
    for (int b = 0; b < B; ++b) {
      pl->h_fin[b] = pl->pending1[b];
      any = any || pl->pending1[b];
    }
    if (!any) return RECON_OK;
    RECON_TRY(full_state());
    RECON_TRY(upload_mask(pl, pl->act_fin, pl->h_fin));
    RECON_TRY(ops->zfinal(pl, pl->psi, nullptr, true, pl->act_fin, false));
    HIP_TRY(pl, hipMemcpyAsync(pl->h_red2.data(), pl->red + 2 * B, 16 * B, hipMemcpyDeviceToHost, pl->stream));
    HIP_TRY(pl, hipStreamSynchronize(pl->stream));
    for (int b = 0; b < B; ++b) {
      if (!pl->pending1[b]) continue;
      pl->psi_valid[b] = 1;
      pl->pending1[b] = 0;
      bool fell = false;
      RECON_TRY(judge_eps1(b, pl->h_red2[2 * b], fell));
    }
    return RECON_OK;
  };

  for (int it = 0; it < max_iter; ++it) {
    Marker mark("a8 correction pass");
    bool any = false;
    for (int b = 0; b < B; ++b) {
      pl->h_it[b] = pl->done[b] ? 0 : 1;
      any = any || pl->h_it[b];
    }
    if (!any) break;
    // realisations that restarted from the plain start need their state X from D_s first
    {
      std::vector<int> want(B, 0);
      bool stale = false;
      for (int b = 0; b < B; ++b) {
        want[b] = pl->h_it[b] && pl->stale_x[b];
        stale = stale || want[b];
      }
      if (stale) RECON_TRY(rebuild_x(want));
    }
    // first: every active realisation is before its first pass (the previous iterate is D_s; a
    // realisation that restarted also holds D_s in D_n).  start_pass: some realisation's first pass
    // from a non-gradient start (all of a plan's realisations reach it together)
    bool first = true, start_pass = false;
    for (int b = 0; b < B; ++b) {
      if (!pl->h_it[b]) continue;
      first = first && pl->passes[b] == 0;
      start_pass = start_pass || (pl->passes[b] == 0 && pl->start_b[b] != RECON_START_PLAIN);
    }
    // eps_1 of a non-gradient start needs S3 = sum Delta u_1; this pass's z step computes u_1
    bool cross = false;
    for (int b = 0; b < B; ++b) cross = cross || (pl->h_it[b] && pl->pending1[b]);
    const int mode = start_pass ? (pl->start == RECON_START_LEARNED ? ZI_LEARNED : ZI_FFTA)
                                : (cross ? ZI_CROSS : ZI_PLAIN);
    // the learned start's pass takes u_p from the start's buffer: it needs no state Y
    const bool need_y = mode != ZI_LEARNED;
    bool any_comb = false, any_fan = false;
    for (int b = 0; b < B; ++b) {
      pl->h_fan[b] = (need_y && pl->h_it[b] && pl->st_y[b] == SY_NONE) ? 1 : 0;
      pl->h_fin[b] = (need_y && pl->h_it[b] && pl->st_y[b] == SY_FULL) ? 1 : 0;   // combined in place
      any_comb = any_comb || pl->h_fin[b];
      any_fan = any_fan || pl->h_fan[b];
    }
    if (any_comb) {
      RECON_TRY(upload_mask(pl, pl->act_fin, pl->h_fin));
      RECON_TRY(ops->combine(pl, pl->act_fin));
    }
    RECON_TRY(upload_mask(pl, pl->act_fan, pl->h_fan));
    RECON_TRY(upload_mask(pl, pl->act_it, pl->h_it));
    const bool steady = mode == ZI_PLAIN && !first;
    const bool graph = steady && (pl->p.flags & RECON_PASS_GRAPHS) && !pl->prof.on;
    if (graph) {
      RECON_TRY(pass_graph_launch(pl, ops));
    } else {
      if (any_fan) RECON_TRY(ops->fanout(pl, pl->act_fan, true));
      RECON_TRY(ops->ziter(pl, mode, pl->act_it));
    }
    if (cross) {
      HIP_TRY(pl, hipMemcpyAsync(pl->h_red2.data(), pl->red + 2 * B, 16 * B, hipMemcpyDeviceToHost, pl->stream));
      HIP_TRY(pl, hipStreamSynchronize(pl->stream));
      bool rest = false;
      for (int b = 0; b < B; ++b) {
        if (!pl->h_it[b] || !pl->pending1[b]) continue;
        pl->pending1[b] = 0;
        bool fell = false;
        RECON_TRY(judge_eps1(b, pl->h_red2[2 * b], fell));
        // a realisation that stops here keeps D_1: its z step is dropped and Psi_1 recomputed at the
        // end; one that restarts from the plain start drops the rest of the pass too
        if (pl->done[b] || fell) {
          pl->h_it[b] = 0;
          if (!fell) {
            pl->st_y[b] = SY_NONE;
            pl->psi_valid[b] = 0;
            pl->stale_x[b] = 1;
          }
        }
      }
      for (int b = 0; b < B; ++b) rest = rest || pl->h_it[b];
      if (!rest) continue;
      RECON_TRY(upload_mask(pl, pl->act_it, pl->h_it));
    }
    // relaxed passes mix with D_n; the first pass after a non-gradient start has no D_0 and is plain
    if (!graph) RECON_TRY(ops->fanin_xiter(pl, first, pl->act_it, start_pass ? 1.f : relax_weight(pl)));
    // the start pass also reads S1, S2 (red[2B..4B)): one copy of both halves
    HIP_TRY(pl, hipMemcpyAsync(pl->h_red.data(), pl->red, (start_pass ? 32 : 16) * B, hipMemcpyDeviceToHost,
                               pl->stream));
    HIP_TRY(pl, hipStreamSynchronize(pl->stream));
    for (int b = 0; b < B; ++b) {
      if (!pl->h_it[b]) continue;
      pl->st_y[b] = SY_NONE;
      pl->psi_valid[b] = 0;
      const bool was_start = pl->passes[b] == 0 && pl->start_b[b] != RECON_START_PLAIN;
      pl->passes[b] += 1;
      const double num = pl->h_red[2 * b], den = pl->h_red[2 * b + 1];
      if (was_start) {
        pl->num0[b] = num * norm_k;
        pl->den0[b] = den * norm_k;
        pl->s1[b] = pl->h_red[2 * B + 2 * b];
        pl->s2[b] = pl->h_red[2 * B + 2 * b + 1];
        pl->pending1[b] = 1;
      } else {
        RECON_TRY(record(b, den > 0 ? std::sqrt(num / den) : 0.0, den * norm_k));
      }
    }
  }
  Marker mark_final("a9 final Psi");
  RECON_TRY(resolve_pending());
  // displacement of every realisation whose Psi buffer is stale (realisations stopped inside a pass
  // get state X again from D_n first)
  bool need = false;
  for (int b = 0; b < B; ++b) {
    pl->h_fin[b] = pl->psi_valid[b] ? 0 : 1;
    need = need || pl->h_fin[b];
  }
  if (need) {
    RECON_TRY(full_state());
    RECON_TRY(upload_mask(pl, pl->act_fin, pl->h_fin));
    RECON_TRY(ops->zfinal(pl, pl->psi, nullptr, false, pl->act_fin, false));
    for (int b = 0; b < B; ++b)
      if (pl->h_fin[b]) pl->psi_valid[b] = 1;
  }
  // the final displacement transform stays queued on the stream: what follows reads host state only
  bool div = false, notconv = false;
  for (int b = 0; b < B; ++b) {
    if (iters_out) iters_out[b] = pl->passes[b];
    if (eps_out)
      for (int i = 0; i < max_iter; ++i)
        eps_out[(size_t)b * max_iter + i] = i < (int)call_eps[b].size() ? call_eps[b][i] : NAN;
    div = div || pl->diverged[b];
    if (!fixed && !pl->diverged[b]) {
      const auto& h = pl->hist[b];
      if (h.empty() || !(h.back() <= tol)) notconv = true;
    }
  }
  if (div) return fail(pl, RECON_EDIVERGED, "convergence norm rose twice in a row or became non-finite");
  if (notconv) return RECON_NOTCONVERGED;
  if (restarted) return fail(pl, RECON_RESTARTED, "a learned start was rejected; restarted from the plain start");
  return RECON_OK;
}

int recon_start_restarts(const recon_plan_t* pl, int32_t* out) {
  if (!pl || !out) return RECON_EINVAL;
  for (int b = 0; b < pl->batch; ++b) out[b] = pl->restarts[b];
  return RECON_OK;
}

int recon_tile_counts(recon_plan_t* pl, int64_t* out) {
  CHECK_PLAN(pl);
  if (!out) return fail(pl, RECON_EINVAL, "NULL output pointer");
  if (pl->state != ST_SOLVED) return fail(pl, RECON_ESTATE, "no solve yet");
  const long long nt = ops_for(pl->n)->nb_z;   // z tiles per realisation
  const int na = pl->randoms ? 2 : 1;
  std::vector<unsigned char> z((size_t)na * pl->batch * nt), m(pl->randoms ? (size_t)pl->batch * nt : 0);
  HIP_TRY(pl, hipMemcpyAsync(z.data(), pl->zflag, z.size(), hipMemcpyDeviceToHost, pl->stream));
  if (pl->randoms) HIP_TRY(pl, hipMemcpyAsync(m.data(), pl->mflag, m.size(), hipMemcpyDeviceToHost, pl->stream));
  HIP_TRY(pl, hipStreamSynchronize(pl->stream));
  for (int b = 0; b < pl->batch; ++b) {
    int64_t c[3] = {0, 0, 0};
    for (long long t = 0; t < nt; ++t) {
      c[0] += z[(size_t)b * nt + t];
      if (pl->randoms) {
        c[1] += z[((size_t)pl->batch + b) * nt + t];
        c[2] += m[(size_t)b * nt + t];
      }
    }
    out[4 * b + 0] = c[0];
    out[4 * b + 1] = pl->randoms ? c[1] : 0;
    out[4 * b + 2] = pl->randoms ? c[2] : nt;
    out[4 * b + 3] = nt;
  }
  return RECON_OK;
}

int recon_shift(recon_plan_t* pl, int which_flags, const float* pos, int64_t n, const int64_t* offsets,
                float* disp_out, float* pos_out) {
  CHECK_PLAN(pl);
  const int which = which_flags & ~RECON_SHIFT_AS_PAINTED;
  const bool as_painted = (which_flags & RECON_SHIFT_AS_PAINTED) != 0;
  if (which != RECON_GAL && which != RECON_RAN) return fail(pl, RECON_EINVAL, "which must be RECON_GAL or RECON_RAN");
  if (pl->state != ST_SOLVED) return fail(pl, RECON_ESTATE, "iterate must precede shift");
  for (int b = 0; b < pl->batch; ++b)
    if (!pl->psi_valid[b]) return fail(pl, RECON_ESTATE, "displacement not computed; call iterate");
  if (n < 0 || (n > 0 && (!pos || !disp_out))) return fail(pl, RECON_EINVAL, "bad catalogue pointers");
  if (pl->batch > 1 && !offsets && n > 0) return fail(pl, RECON_EINVAL, "offsets are required when batch > 1");
  // the brick-ordered copy is used only when the caller says the catalogue is the one painted last
  // (unchanged since); the call must then name that paint's catalogue
  if (as_painted && !(which == pl->srt_which && pos == pl->srt_pos && n == pl->srt_n && offsets == pl->srt_off))
    return fail(pl, RECON_EINVAL, "RECON_SHIFT_AS_PAINTED: not the catalogue painted last through the bricks");
  if (n == 0) return RECON_OK;
  Marker mark(which == RECON_GAL ? "a10 shift (galaxies)" : "a10 shift (randoms)");
  HIP_TRY(pl, hipMemsetAsync(pl->err + 2, 0, sizeof(int), pl->stream));
  long long blocks = (n + kThreads - 1) / kThreads;
  if (blocks > 8192) blocks = 8192;
  if (as_painted) {
    // the catalogue painted last through the bricks: shift its brick-ordered copy, then reorder
    {
      PROF(pl, KP_SHIFT);
      k_shift_brick<512><<<(unsigned)pl->L.nbins, 512, 0, pl->stream>>>(
          pl->sorted, pl->bstart, pl->psi, pl->cic, (float)pl->p.observer[0], (float)pl->p.observer[1],
          (float)pl->p.observer[2], (float)pl->p.growth, which == RECON_GAL ? 1 : 0, pl->stmp);
      // one trip per block: per XCD, ceil(chunks / 8) chunks of 256 objects in groups of kObjBatch
      const long long chunks = (n + kThreads - 1) / kThreads;
      const long long ub = 8 * (((chunks + 7) / 8 + kObjBatch - 1) / kObjBatch);
      k_shift_unpermute<<<(unsigned)ub, kThreads, 0, pl->stream>>>(
          pl->slot_of, pl->stmp, n, pos, disp_out, pos_out, pl->err + 2);
    }
    return check_launch(pl, "shift (brick order)");
  }
  {
    PROF(pl, KP_SHIFT);
    k_shift<<<(unsigned)blocks, kThreads, 0, pl->stream>>>(
        pos, n, (const long long*)offsets, pl->batch, pl->psi, pl->cic, (float)pl->p.observer[0],
        (float)pl->p.observer[1], (float)pl->p.observer[2], (float)pl->p.growth, which == RECON_GAL ? 1 : 0,
        disp_out, pos_out, pl->err + 2);
  }
  return check_launch(pl, "shift");
}

int recon_get_psi(recon_plan_t* pl, float* psi_out) {
  CHECK_PLAN(pl);
  if (!psi_out) return fail(pl, RECON_EINVAL, "NULL output pointer");
  if (pl->state != ST_SOLVED) return fail(pl, RECON_ESTATE, "no displacement yet");
  for (int b = 0; b < pl->batch; ++b)
    if (!pl->psi_valid[b]) return fail(pl, RECON_ESTATE, "displacement not computed; call iterate");
  // the plan keeps the displacement in the output's layout
  HIP_TRY(pl, hipMemcpyAsync(psi_out, pl->psi, sizeof(float) * 3 * (size_t)pl->n3 * pl->batch,
                             hipMemcpyDeviceToDevice, pl->stream));
  return RECON_OK;
}

int recon_get_grid(recon_plan_t* pl, int which, int64_t* out) {
  CHECK_PLAN(pl);
  if (!out) return fail(pl, RECON_EINVAL, "NULL output pointer");
  if (which != RECON_GAL && which != RECON_RAN) return fail(pl, RECON_EINVAL, "which must be RECON_GAL or RECON_RAN");
  const long long* g = which == RECON_GAL ? pl->grid_g : pl->grid_r;
  if (!g || !(which == RECON_GAL ? pl->painted_g : pl->painted_r)) return fail(pl, RECON_ESTATE, "grid not painted");
  if (const unsigned char* v = valid_of(pl, which)) {
    long long blocks = (pl->n3 * pl->batch + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    k_grid_export<<<(unsigned)blocks, 256, 0, pl->stream>>>(g, v, pl->n, pl->batch, (long long*)out);
    return check_launch(pl, "grid export");
  }
  HIP_TRY(pl, hipMemcpyAsync(out, g, sizeof(int64_t) * pl->n3 * pl->batch, hipMemcpyDeviceToDevice, pl->stream));
  return RECON_OK;
}

int recon_radial_ratio(recon_plan_t* pl, const float* psi_ref, double lo, double hi, double* stats_out) {
  CHECK_PLAN(pl);
  if (!psi_ref || !stats_out) return fail(pl, RECON_EINVAL, "NULL pointer");
  if (!(lo <= hi)) return fail(pl, RECON_EINVAL, "need lo <= hi");
  if (pl->state != ST_SOLVED) return fail(pl, RECON_ESTATE, "no displacement yet");
  for (int b = 0; b < pl->batch; ++b)
    if (!pl->psi_valid[b]) return fail(pl, RECON_ESTATE, "displacement not computed; call iterate");
  constexpr int NT = 256;
  long long blocks = (pl->n3 + NT - 1) / NT;
  if (blocks > 1024) blocks = 1024;
  k_ratio_stats<NT><<<dim3((unsigned)blocks, pl->batch), NT, 0, pl->stream>>>(
      pl->psi, psi_ref, pl->geo, pl->n, lo, hi, pl->partials, pl->tpart);
  RECON_TRY(check_launch(pl, "radial ratio"));
  std::vector<double> part(2 * blocks * pl->batch);
  std::vector<unsigned long long> cnt(blocks * pl->batch);
  HIP_TRY(pl, hipMemcpyAsync(part.data(), pl->partials, part.size() * 8, hipMemcpyDeviceToHost, pl->stream));
  HIP_TRY(pl, hipMemcpyAsync(cnt.data(), pl->tpart, cnt.size() * 8, hipMemcpyDeviceToHost, pl->stream));
  HIP_TRY(pl, hipStreamSynchronize(pl->stream));
  for (int b = 0; b < pl->batch; ++b) {
    double s1 = 0.0, s2 = 0.0;
    unsigned long long c = 0;
    for (long long k = 0; k < blocks; ++k) {
      s1 += part[2 * (b * blocks + k)];
      s2 += part[2 * (b * blocks + k) + 1];
      c += cnt[b * blocks + k];
    }
    const double mean = c ? s1 / (double)c : 0.0;
    const double var = c ? std::fmax(s2 / (double)c - mean * mean, 0.0) : 0.0;
    stats_out[4 * b + 0] = mean;
    stats_out[4 * b + 1] = std::sqrt(var);
    stats_out[4 * b + 2] = 1.0 - (double)c / (double)pl->n3;
    stats_out[4 * b + 3] = (double)c;
  }
  return RECON_OK;
}

int recon_helmholtz(recon_plan_t* pl, const float* psi_x, float* irr_out, float* sol_out) {
  CHECK_PLAN(pl);
  if (!psi_x || !irr_out) return fail(pl, RECON_EINVAL, "NULL pointer");
  const Ops* ops = ops_for(pl->n);
  RECON_TRY(ops->helm(pl, psi_x));
  for (int b = 0; b < pl->batch; ++b) pl->h_fan[b] = 1;
  RECON_TRY(upload_mask(pl, pl->act_fan, pl->h_fan));
  RECON_TRY(ops->fanout(pl, pl->act_fan, false));
  RECON_TRY(upload_mask(pl, pl->act_fin, pl->h_fan));
  RECON_TRY(ops->zfinal(pl, pl->psi, nullptr, false, pl->act_fin, false));
  long long nb = (pl->n3 * pl->batch + 255) / 256;
  if (nb > 65536) nb = 65536;
  k_helm_out<<<(unsigned)nb, 256, 0, pl->stream>>>(pl->psi, psi_x, pl->n, pl->batch, irr_out, sol_out);
  RECON_TRY(check_launch(pl, "Helmholtz output"));
  // the transform buffers, D_s and Psi now hold the diagnostic: the reconstruction starts over
  pl->state = ST_EMPTY;
  pl->painted_g = pl->painted_r = false;
  for (int b = 0; b < pl->batch; ++b) {
    pl->psi_valid[b] = 0;
    pl->st_y[b] = 0;
  }
  return RECON_OK;
}

int recon_get_delta(recon_plan_t* pl, float* out) {
  CHECK_PLAN(pl);
  if (!out) return fail(pl, RECON_EINVAL, "NULL output pointer");
  if (!pl->delta) return fail(pl, RECON_EINVAL, "plan was created without RECON_KEEP_DELTA");
  if (pl->state != ST_SOLVED && pl->state != ST_DELTA) return fail(pl, RECON_ESTATE, "no overdensity yet");
  HIP_TRY(pl, hipMemcpyAsync(out, pl->delta, sizeof(float) * pl->n3 * pl->batch, hipMemcpyDeviceToDevice, pl->stream));
  return RECON_OK;
}

int recon_cnn_forward(recon_plan_t* pl, const float* params, const float* delta, const float* u_p, float* du_out) {
  CHECK_PLAN(pl);
  if (!pl->a1) return fail(pl, RECON_EINVAL, "plan was created without RECON_CNN_BUFFERS");
  if (!params || !delta || !u_p || !du_out) return fail(pl, RECON_EINVAL, "NULL pointer");
  return cnn_forward_impl(pl, params, delta, u_p, du_out, 1.0f / recon::cnn::S_U);
}

int recon_cnn_train_step(recon_plan_t* pl, float* params, float* adam_m, float* adam_v, int step, float lr,
                         const float* delta, const float* u_p, const float* target_du, double* loss_out,
                         float* grad_out) {
  using namespace recon::cnn;
  CHECK_PLAN(pl);
  if (!pl->a1) return fail(pl, RECON_EINVAL, "plan was created without RECON_CNN_BUFFERS");
  if (!params || !delta || !u_p || !target_du) return fail(pl, RECON_EINVAL, "NULL pointer");
  if (lr > 0.f && (!adam_m || !adam_v || step < 1)) return fail(pl, RECON_EINVAL, "Adam needs moments and step >= 1");
  const long long count = pl->cnn_n3 * pl->batch;
  RECON_TRY(cnn_forward_impl(pl, params, delta, u_p, pl->ybuf, 1.0f));
  const dim3 grid((unsigned)pl->L.nb_conv, pl->batch);
  const dim3 gridw((unsigned)pl->L.nb_w, pl->batch);
  const Geo3 g = cnn_geo(pl);
  hipStream_t s = pl->stream;
  {
    PROF(pl, KP_CNN_BWD);
    k_loss<<<(unsigned)pl->L.nb_loss, 256, 0, s>>>(pl->ybuf, target_du, count, pl->dybuf, pl->lossp);
    k_conv_out_bwd<<<grid, 256, 0, s>>>(pl->dybuf, pl->a2, g, pl->w3, pl->d2, pl->part_out);
    k_wgrad16<CH, K2, 0><<<gridw, 256, 0, s>>>(pl->d2, pl->a1, nullptr, nullptr, g, pl->part_w2);
    k_conv16<CH, K2, 0, 1><<<grid, 256, 0, s>>>(pl->d2, nullptr, nullptr, g, pl->wk2t, nullptr, pl->a1, pl->d1);
    k_wgrad16<CIN, K1P, 1><<<gridw, 256, 0, s>>>(pl->d1, nullptr, delta, u_p, g, pl->part_w1);
    const long long nbo = pl->L.nb_conv * pl->batch, nbw = pl->L.nb_w * pl->batch;
    k_reduce_cols<<<(K2 + 1 + 255) / 256, 256, 0, s>>>(pl->part_out, nbo, K2 + 1, pl->g3);
    k_reduce_cols<<<(CH * (K2 + 1) + 255) / 256, 256, 0, s>>>(pl->part_w2, nbw, CH * (K2 + 1), pl->g2);
    k_reduce_cols<<<(CH * (K1P + 1) + 255) / 256, 256, 0, s>>>(pl->part_w1, nbw, CH * (K1P + 1), pl->g1);
    float* grad = grad_out ? grad_out : pl->gradbuf;
    k_assemble_grad<<<(NPARAM + 255) / 256, 256, 0, s>>>(pl->g1, pl->g2, pl->g3, grad);
    k_reduce_loss<<<1, 256, 0, s>>>(pl->lossp, (int)pl->L.nb_loss, pl->losst);
    if (lr > 0.f) {
      const float c1 = (float)(1.0 - std::pow(0.9, step)), c2 = (float)(1.0 - std::pow(0.999, step));
      k_adam<<<(NPARAM + 255) / 256, 256, 0, s>>>(params, adam_m, adam_v, grad, NPARAM, lr, 0.9f, 0.999f, 1e-8f,
                                                  c1, c2);
    }
  }
  RECON_TRY(check_launch(pl, "network training step"));
  double lsum = 0.0;
  HIP_TRY(pl, hipMemcpyAsync(&lsum, pl->losst, 8, hipMemcpyDeviceToHost, s));
  HIP_TRY(pl, hipStreamSynchronize(s));
  if (loss_out) *loss_out = lsum / (double)count;
  return RECON_OK;
}

int recon_get_radial(recon_plan_t* pl, float* u_out) {
  CHECK_PLAN(pl);
  if (!u_out) return fail(pl, RECON_EINVAL, "NULL output pointer");
  if (pl->state != ST_SOLVED) return fail(pl, RECON_ESTATE, "no displacement yet");
  for (int b = 0; b < pl->batch; ++b)
    if (!pl->psi_valid[b]) return fail(pl, RECON_ESTATE, "displacement not computed; call iterate");
  long long blocks = (pl->n3 * pl->batch + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  recon::cnn::k_radial<<<(unsigned)blocks, 256, 0, pl->stream>>>(pl->psi, grid_geo(pl, false), pl->batch, u_out);
  return check_launch(pl, "radial component");
}

int recon_restrict(recon_plan_t* pl, const float* fine, float* coarse) {
  CHECK_PLAN(pl);
  if (!fine || !coarse) return fail(pl, RECON_EINVAL, "NULL pointer");
  return restrict_impl(pl, fine, coarse);
}

int recon_prolong(recon_plan_t* pl, const float* coarse, float* fine) {
  CHECK_PLAN(pl);
  if (!coarse || !fine) return fail(pl, RECON_EINVAL, "NULL pointer");
  return prolong_impl(pl, coarse, 1.0f, fine);
}

int recon_profile_start(recon_plan_t* pl) {
  if (!pl) return RECON_EINVAL;
  pl->prof.on = true;
  pl->prof.used = 0;
  pl->prof.recs.clear();
  return RECON_OK;
}

int recon_profile_stop(recon_plan_t* pl, int32_t* counts, double* total_ms, int cap) {
  if (!pl) return RECON_EINVAL;
  pl->prof.on = false;
  HIP_TRY(pl, hipStreamSynchronize(pl->stream));
  std::vector<int32_t> c(KP_COUNT, 0);
  std::vector<double> t(KP_COUNT, 0.0);
  for (const auto& r : pl->prof.recs) {
    float ms = 0.f;
    HIP_TRY(pl, hipEventElapsedTime(&ms, pl->prof.pool[r.second], pl->prof.pool[r.second + 1]));
    c[r.first] += 1;
    t[r.first] += ms;
  }
  pl->prof.recs.clear();
  pl->prof.used = 0;
  for (int k = 0; k < KP_COUNT && k < cap; ++k) {
    if (counts) counts[k] = c[k];
    if (total_ms) total_ms[k] = t[k];
  }
  return KP_COUNT;
}

int64_t recon_debug_violations(int reset) {
#ifdef RECON_DEBUG
  if (hipDeviceSynchronize() != hipSuccess) return -2;
  unsigned long long v = 0;
  if (hipMemcpyFromSymbol(&v, HIP_SYMBOL(recon::recon_debug_count), sizeof v, 0, hipMemcpyDeviceToHost) != hipSuccess)
    return -2;
  if (reset) {
    const unsigned long long z = 0;
    if (hipMemcpyToSymbol(HIP_SYMBOL(recon::recon_debug_count), &z, sizeof z, 0, hipMemcpyHostToDevice) != hipSuccess)
      return -2;
  }
  return (int64_t)v;
#else
  (void)reset;
  return -1;
#endif
}

const char* recon_profile_kernel_name(int id) {
  return (id >= 0 && id < KP_COUNT) ? kKernelNames[id] : "";
}

}  // extern "C"
