// The batched form: many independent instances of uneven sizes (A_i *_Q_i B_i
// and the truncated tSVDQ of A_i, Def. 3.1 and Alg. 4.1) in one captured
// graph.  The transforms and back-projections of all instances run as
// grouped launches over tables of strips (one per vector width); the
// facewise products of all instances run as one grouped GEMM launch over a
// table of 128 x 128 output tiles; the Jacobi sweeps, which dominate, run as
// grouped launches over the faces of every instance at once (a device table
// of face offsets and sizes, and per-round lists of the block-pair visits
// that exist, so that a launch has no workgroup for a face without a visit
// in that round); the finishing steps run as grouped launches over a table
// of every face's operands.  The plan call runs the whole batch once eagerly
// (the outputs of that run are valid; new launch shapes are tuned there
// while tuning is on), then captures the same launch sequence on a private
// stream into a hipGraph; pq_batched_run replays it with one hipGraphLaunch.
#include <algorithm>
#include <cstdint>
#include <new>
#include <vector>

#include "../../include/projprod.h"
#include "internal.hpp"

struct pq_batch_s {
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

namespace {

constexpr size_t kAlign = 256;
size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }
constexpr int kMaxSweepsCap = 100;
constexpr int kDefaultSweeps = 10;
constexpr double kCoarseTol = 1e-5;
constexpr int kPolishSweeps = 6;
constexpr int kTopPolishSweeps = 4;  // the top-block polish: 1-2 sweeps from the float32 stop
constexpr double kTolFloor = 1e-10;
constexpr double kDefaultTol = 1e-13;
constexpr int64_t kMaxLen = 512;  // longest Jacobi vector of a batched tSVDQ face

int hip_rc(hipError_t e) { return e == hipSuccess ? PQ_OK : pq::note_hip_error(e); }

#define BQ_TRY(expr)                         \
  do {                                       \
    int _rc = hip_rc(expr);                  \
    if (_rc != PQ_OK) return _rc;            \
  } while (0)
#define BQ_CHECK(expr)                       \
  do {                                       \
    int _rc = (expr);                        \
    if (_rc != PQ_OK) return _rc;            \
  } while (0)

bool has_svd(const pq_instance& x) { return x.Uhat != nullptr; }

// Workspace layout of a batch (byte offsets into the caller's workspace).
struct Layout {
  size_t faces = 0;            // JFace table (device)
  std::vector<size_t> ah;      // per instance: Ah (float32, n1 x n2 x p)
  std::vector<size_t> bh, ch;  // per product instance: Bh (n2 x n4 x p), Ch (n1 x n4 x p)
  size_t gdesc = 0, gtile = 0;  // grouped facewise GEMM: product and tile tables
  int nprod = 0, ntiles = 0;
  // grouped transforms: descriptors (forward ones first), forward and return
  // tile tables (sized for one tube per lane, the most tiles)
  size_t xdesc = 0, htile = 0, utile = 0;
  int nxdesc = 0;
  int64_t hmax = 0, umax = 0;
  std::vector<int64_t> woff;   // per instance: element offset of its faces in W32 / W64
  std::vector<int> face0;      // per instance: index of its first face
  size_t w32 = 0, w64 = 0, used1 = 0, used2 = 0, flags = 0;
  std::vector<size_t> sig, ft, y, ys;  // per instance finishing buffers
  size_t total = 0;
  int nfaces = 0, nb_max = 2, L_max = 1;
  int nv_max = 1;
  size_t tnrm = 0, tpos = 0;  // top-block norms and positions, nfaces x nv_max
  size_t fin = 0;             // finishing table (FinFace per face)
  pq::FinMax fmax;
  int ntop = 2;  // leading blocks of the top-block polish (0: every pair)
  int64_t welems = 0;
  std::vector<pq::JFace> tab;  // host copy of the face table
  // per-round visit lists of the float32 sweeps (every pair) and of the
  // float64 polish (top-block schedule), host copies and device offsets
  std::vector<int> v32, off32, v64, off64;
  size_t dv32 = 0, dv64 = 0;
  // the float32 lists of the parts of the faces (faces dealt in turn in
  // order of vector length) for the sweeps on several streams
  std::vector<int> v32p[pq::kSweepParts], off32p[pq::kSweepParts];
  std::vector<int> v64p[pq::kSweepParts], off64p[pq::kSweepParts];
  size_t dv32p[pq::kSweepParts] = {}, dv64p[pq::kSweepParts] = {};
  bool listed = false;
};

int validate(const pq_instance* inst, int count) {
  if (!inst) return PQ_ERR_NULL;
  if (count < 1) return PQ_ERR_ARG;
  for (int i = 0; i < count; ++i) {
    const pq_instance& x = inst[i];
    if (!x.A || !x.Q) return PQ_ERR_NULL;
    for (int64_t d : {x.n1, x.n2, x.n3, x.p})
      if (d < 1) return PQ_ERR_SHAPE;
    if (x.p > x.n3) return PQ_ERR_P;
    if (x.p > 512 || x.n1 * x.n2 >= ((int64_t)1 << 31)) return PQ_ERR_UNSUPPORTED;
    if ((x.B == nullptr) != (x.C == nullptr)) return PQ_ERR_NULL;
    if (x.B && x.n4 < 1) return PQ_ERR_SHAPE;
    if (x.B && x.n1 * x.n4 >= ((int64_t)1 << 31)) return PQ_ERR_UNSUPPORTED;
    const bool svd = has_svd(x);
    if (svd != (x.s != nullptr) || svd != (x.Vhat != nullptr)) return PQ_ERR_NULL;
    if (!x.B && !svd) return PQ_ERR_ARG;  // nothing to compute
    if (svd) {
      if (x.k < 1 || x.k > std::min(x.n1, x.n2)) return PQ_ERR_K;
      if (std::max(x.n1, x.n2) > kMaxLen) return PQ_ERR_UNSUPPORTED;
    }
    for (const void* o : {(const void*)x.C, (const void*)x.Uhat, (const void*)x.s, (const void*)x.Vhat})
      if (o && (o == x.A || o == x.B || o == x.Q)) return PQ_ERR_ALIAS;
  }
  return PQ_OK;
}

Layout layout(const pq_instance* inst, int count) {
  Layout lo;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off += align_up(bytes);
    return o;
  };
  lo.ah.resize(count);
  lo.woff.assign(count, 0);
  lo.face0.assign(count, 0);
  lo.sig.assign(count, 0);
  lo.ft.assign(count, 0);
  lo.y.assign(count, 0);
  lo.ys.assign(count, 0);
  for (int i = 0; i < count; ++i) {
    const pq_instance& x = inst[i];
    if (x.B)
    {
      ++lo.nprod;
      lo.ntiles += (int)(((x.n1 + 127) / 128) * ((x.n4 + 127) / 128) * x.p);
    }
    if (has_svd(x)) {
      lo.face0[i] = lo.nfaces;
      lo.woff[i] = lo.welems;
      lo.nfaces += (int)x.p;
      lo.welems += x.n1 * x.n2 * x.p;
      const int nv = (int)std::min(x.n1, x.n2);
      int nb = (nv + 15) / 16;
      nb += nb & 1;
      lo.nb_max = std::max(lo.nb_max, nb);
      lo.L_max = std::max(lo.L_max, (int)std::max(x.n1, x.n2));
      lo.nv_max = std::max(lo.nv_max, nv);
      lo.fmax.n1 = std::max(lo.fmax.n1, (int)x.n1);
      lo.fmax.n2 = std::max(lo.fmax.n2, (int)x.n2);
      lo.fmax.nv = std::max(lo.fmax.nv, nv);
      lo.fmax.nvL = std::max(lo.fmax.nvL, (int)(x.n1 + x.n2));
      lo.fmax.kr = std::max(lo.fmax.kr, pq::ritz_cols(x.k, nv));
      // enough leading blocks for every instance's Ritz columns
      const int tb = pq::top_blocks(pq::ritz_cols(x.k, nv));
      lo.ntop = (tb == 0 || lo.ntop == 0) ? 0 : std::max(lo.ntop, tb);
    }
  }
  lo.faces = take(sizeof(pq::JFace) * std::max(1, lo.nfaces));
  // the face table: every face of every tSVDQ instance, in order, and the
  // sweeps' visit lists over it
  lo.tab.reserve(lo.nfaces);
  for (int i = 0; i < count; ++i) {
    const pq_instance& x = inst[i];
    if (!has_svd(x)) continue;
    const int nv = (int)std::min(x.n1, x.n2), L = (int)std::max(x.n1, x.n2);
    for (int64_t l = 0; l < x.p; ++l) lo.tab.push_back(pq::JFace{lo.woff[i] + l * nv * L, nv, L});
  }
  std::vector<char> pick[pq::kSweepParts];
  {
    std::vector<int> order((size_t)lo.nfaces);
    for (int f = 0; f < lo.nfaces; ++f) order[(size_t)f] = f;
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return lo.tab[a].L > lo.tab[b].L; });
    for (int k = 0; k < pq::kSweepParts; ++k) pick[k].assign((size_t)lo.nfaces, 0);
    for (size_t r = 0; r < order.size(); ++r) pick[r % pq::kSweepParts][(size_t)order[r]] = 1;
  }
  lo.listed = pq::jacobi_visit_list(lo.tab.data(), lo.nfaces, 0, lo.v32, lo.off32) &&
              pq::jacobi_visit_list(lo.tab.data(), lo.nfaces, lo.ntop, lo.v64, lo.off64);
  for (int k = 0; k < pq::kSweepParts && lo.listed; ++k)
    lo.listed = pq::jacobi_visit_list(lo.tab.data(), lo.nfaces, 0, lo.v32p[k], lo.off32p[k], &pick[k]) &&
                pq::jacobi_visit_list(lo.tab.data(), lo.nfaces, lo.ntop, lo.v64p[k], lo.off64p[k], &pick[k]);
  lo.dv32 = take(sizeof(int) * std::max<size_t>(1, lo.v32.size()));
  lo.dv64 = take(sizeof(int) * std::max<size_t>(1, lo.v64.size()));
  for (int k = 0; k < pq::kSweepParts; ++k) {
    lo.dv32p[k] = take(sizeof(int) * std::max<size_t>(1, lo.v32p[k].size()));
    lo.dv64p[k] = take(sizeof(int) * std::max<size_t>(1, lo.v64p[k].size()));
  }
  for (int i = 0; i < count; ++i) lo.ah[i] = take(4 * (size_t)inst[i].n1 * inst[i].n2 * inst[i].p);
  lo.bh.assign(count, 0);
  lo.ch.assign(count, 0);
  for (int i = 0; i < count; ++i) {
    const pq_instance& x = inst[i];
    if (!x.B) continue;
    lo.bh[i] = take(4 * (size_t)x.n2 * x.n4 * x.p);
    lo.ch[i] = take(4 * (size_t)x.n1 * x.n4 * x.p);
  }
  for (int i = 0; i < count; ++i) {
    const pq_instance& x = inst[i];
    const int chunks = (int)((x.p + 31) / 32);
    lo.hmax += (x.n1 * x.n2 + 31) / 32 * chunks;
    ++lo.nxdesc;
    if (x.B) {
      lo.hmax += (x.n2 * x.n4 + 31) / 32 * chunks;
      ++lo.nxdesc;
      if (x.p <= 32) {
        lo.umax += ((x.n1 * x.n4 + 31) / 32 + 3) / 4;
        ++lo.nxdesc;
      }
    }
  }
  lo.xdesc = take(sizeof(pq::XformDesc) * (size_t)lo.nxdesc);
  lo.htile = take(sizeof(pq::XformTile) * (size_t)std::max<int64_t>(1, lo.hmax));
  lo.utile = take(sizeof(pq::XformTile) * (size_t)std::max<int64_t>(1, lo.umax));
  lo.gdesc = take(sizeof(pq::GemmDesc) * (size_t)std::max(1, lo.nprod));
  lo.gtile = take(sizeof(pq::GemmTile) * (size_t)std::max(1, lo.ntiles));
  lo.w32 = take(4 * (size_t)std::max<int64_t>(lo.welems, 1));
  lo.w64 = take(8 * (size_t)std::max<int64_t>(lo.welems, 1));
  lo.used1 = take(sizeof(int) * std::max(1, lo.nfaces));
  lo.used2 = take(sizeof(int) * std::max(1, lo.nfaces));
  lo.flags = take(sizeof(int) * (size_t)std::max(1, lo.nfaces) * kMaxSweepsCap);
  lo.tnrm = take(sizeof(double) * (size_t)std::max(1, lo.nfaces) * lo.nv_max);
  lo.tpos = take(sizeof(int) * (size_t)std::max(1, lo.nfaces) * lo.nv_max);
  lo.fin = take(sizeof(pq::FinFace) * (size_t)std::max(1, lo.nfaces));
  for (int i = 0; i < count; ++i) {
    const pq_instance& x = inst[i];
    if (!has_svd(x)) continue;
    const size_t mx = std::max(x.n1, x.n2), mn = std::min(x.n1, x.n2);
    const size_t kr = (size_t)pq::ritz_cols(x.k, (int64_t)mn);
    lo.sig[i] = take(8 * mn * x.p);
    lo.ft[i] = take(8 * mx * kr * x.p);
    lo.y[i] = take(8 * mn * kr * x.p);
    lo.ys[i] = take(4 * mn * x.k * x.p);
  }
  lo.total = off;
  return lo;
}

// Enqueue every launch of the batch on s.
// host side of the grouped transforms: tiles of the forward and return
// transforms by vector width (index 0: two tubes per lane, 1: one)
struct XformPlan {
  int nh[3] = {0, 0, 0}, nu[3] = {0, 0, 0};  // by tubes per lane: 4, 2, 1
  size_t uq[3] = {0, 0, 0};                  // largest Q of each return group, staged in LDS (bytes)
};

int enqueue(const Layout& lo, const pq_instance* inst, int count, int max_sweeps, double tol, int* info_dev,
            char* ws, const XformPlan& xp, hipStream_t s, const pq::SweepPair* pair) {
  float* W32 = reinterpret_cast<float*>(ws + lo.w32);
  double* W64 = reinterpret_cast<double*>(ws + lo.w64);
  int* used1 = reinterpret_cast<int*>(ws + lo.used1);
  int* used2 = reinterpret_cast<int*>(ws + lo.used2);
  int* flags = reinterpret_cast<int*>(ws + lo.flags);
  const pq::JFace* faces = reinterpret_cast<const pq::JFace*>(ws + lo.faces);
  // the transforms of every instance, the facewise products and the
  // back-projections, one launch each (per vector width)
  const pq::XformDesc* xd = reinterpret_cast<const pq::XformDesc*>(ws + lo.xdesc);
  const pq::XformTile* ht = reinterpret_cast<const pq::XformTile*>(ws + lo.htile);
  const pq::XformTile* ut = reinterpret_cast<const pq::XformTile*>(ws + lo.utile);
  {
    pq::ProfScope prof("hat", s, (xp.nh[0] > 0) + (xp.nh[1] > 0) + (xp.nh[2] > 0));
    BQ_TRY(pq::hat_grouped(xd, ht, xp.nh[0], 4, s));
    BQ_TRY(pq::hat_grouped(xd, ht + xp.nh[0], xp.nh[1], 2, s));
    BQ_TRY(pq::hat_grouped(xd, ht + xp.nh[0] + xp.nh[1], xp.nh[2], 1, s));
  }
  if (lo.ntiles > 0) {
    pq::ProfScope prof("facewise_gemm", s);
    BQ_TRY(pq::gemm_f32_grouped(reinterpret_cast<const pq::GemmDesc*>(ws + lo.gdesc),
                                reinterpret_cast<const pq::GemmTile*>(ws + lo.gtile), lo.ntiles, s));
  }
  {
    pq::ProfScope prof("unhat", s, (xp.nu[0] > 0) + (xp.nu[1] > 0) + (xp.nu[2] > 0));
    BQ_TRY(pq::unhat_grouped(xd, ut, xp.nu[0], 4, xp.uq[0], s));
    BQ_TRY(pq::unhat_grouped(xd, ut + xp.nu[0], xp.nu[1], 2, xp.uq[1], s));
    BQ_TRY(pq::unhat_grouped(xd, ut + xp.nu[0] + xp.nu[1], xp.nu[2], 1, xp.uq[2], s));
  }
  for (int i = 0; i < count; ++i) {  // products of more than 32 faces
    const pq_instance& x = inst[i];
    if (x.B && x.p > 32)
      BQ_CHECK(pq_unhat(ws + lo.ch[i], x.Q, x.C, PQ_F32, x.n1, x.n4, x.n3, x.p, PQ_PREC_DEFAULT, s));
  }
  if (lo.nfaces == 0) return PQ_OK;
  // Jacobi vectors of every face, then the grouped sweeps
  for (int i = 0; i < count; ++i) {
    const pq_instance& x = inst[i];
    if (!has_svd(x)) continue;
    BQ_TRY(pq::jacobi_prep_f32(reinterpret_cast<const float*>(ws + lo.ah[i]), W32 + lo.woff[i], (int)x.n1,
                               (int)x.n2, (int)x.p, s));
  }
  const pq::VisitList vl32{reinterpret_cast<const int*>(ws + lo.dv32), lo.off32.data()};
  const pq::VisitList vl64{reinterpret_cast<const int*>(ws + lo.dv64), lo.off64.data()};
  pq::VisitList vl32p[pq::kSweepParts], vl64p[pq::kSweepParts];
  pq::SweepPair sp, sp64;
  if (pair && lo.listed) {
    sp = sp64 = *pair;
    for (int k = 0; k < pq::kSweepParts; ++k) {
      vl32p[k] = pq::VisitList{reinterpret_cast<const int*>(ws + lo.dv32p[k]), lo.off32p[k].data()};
      vl64p[k] = pq::VisitList{reinterpret_cast<const int*>(ws + lo.dv64p[k]), lo.off64p[k].data()};
      sp.vl[k] = &vl32p[k];
      sp64.vl[k] = &vl64p[k];
    }
  }
  BQ_TRY(pq::jacobi_gram_grouped_f32(W32, faces, lo.nfaces, lo.nb_max, lo.L_max, max_sweeps, kCoarseTol,
                                     lo.ntop > 0 ? pq::kCoarseStop32 : kCoarseTol, used1,
                                     flags, lo.listed ? &vl32 : nullptr, s, pair && lo.listed ? &sp : nullptr));
  if (lo.ntop > 0)
    BQ_TRY(pq::jacobi_widen_top(W32, W64, faces, lo.nfaces, 0, 0, lo.nv_max, 16 * lo.ntop,
                                reinterpret_cast<double*>(ws + lo.tnrm), reinterpret_cast<int*>(ws + lo.tpos), s));
  else
    BQ_TRY(pq::jacobi_widen(W32, W64, lo.welems, s));
  const int polish = std::min(max_sweeps, lo.ntop > 0 ? kTopPolishSweeps : kPolishSweeps);
  const double ptol = std::max(tol, kTolFloor);
  BQ_TRY(pq::jacobi_gram_grouped_f64(W64, faces, lo.nfaces, lo.nb_max, lo.L_max, polish, ptol,
                                     lo.ntop > 0 ? pq::kPolishStop32 : ptol, lo.ntop, used2, flags,
                                     lo.listed ? &vl64 : nullptr, s, pair && lo.listed ? &sp64 : nullptr));
  // finishing of every face at once: the top kr vectors, the other factor
  // and the Ritz step (one launch each over the face table)
  BQ_TRY(pq::jacobi_finish_grouped(reinterpret_cast<const pq::FinFace*>(ws + lo.fin), lo.nfaces, lo.fmax, tol, s));
  if (info_dev) BQ_TRY(pq::jacobi_info(used1, used2, lo.nfaces, max_sweeps, polish, info_dev, s));
  return PQ_OK;
}

}  // namespace

extern "C" {

int pq_batched_workspace(const pq_instance* inst, int count, size_t* bytes) {
  if (!bytes) return PQ_ERR_NULL;
  BQ_CHECK(validate(inst, count));
  *bytes = layout(inst, count).total;
  return PQ_OK;
}

int pq_batched_plan(const pq_instance* inst, int count, int max_sweeps, double tol, int* info_dev, void* ws,
                    size_t ws_bytes, hipStream_t stream, pq_batch* out) {
  if (!out || !ws) return PQ_ERR_NULL;
  *out = nullptr;
  BQ_CHECK(validate(inst, count));
  if (max_sweeps <= 0) max_sweeps = kDefaultSweeps;
  if (max_sweeps > kMaxSweepsCap) return PQ_ERR_ARG;
  if (tol <= 0.0) tol = kDefaultTol;
  const Layout lo = layout(inst, count);
  if (ws_bytes < lo.total) return PQ_ERR_WORKSPACE;
  char* w = static_cast<char*>(ws);
  // the finishing table: every face's operands and outputs
  std::vector<pq::FinFace> fin;
  fin.reserve(lo.nfaces);
  double* W64 = reinterpret_cast<double*>(w + lo.w64);
  for (int i = 0; i < count; ++i) {
    const pq_instance& x = inst[i];
    if (!has_svd(x)) continue;
    const bool cols = x.n1 >= x.n2;
    const int64_t nv = std::min(x.n1, x.n2), L = std::max(x.n1, x.n2);
    const int64_t kr = pq::ritz_cols(x.k, nv);
    float* Fo = static_cast<float*>(cols ? x.Uhat : x.Vhat);
    float* Other = static_cast<float*>(cols ? x.Vhat : x.Uhat);
    for (int64_t l = 0; l < x.p; ++l) {
      pq::FinFace f;
      f.w = W64 + lo.woff[i] + l * nv * L;
      f.ah = reinterpret_cast<const float*>(w + lo.ah[i]) + l * x.n1 * x.n2;
      f.sig = reinterpret_cast<double*>(w + lo.sig[i]) + l * nv;
      f.ft = reinterpret_cast<double*>(w + lo.ft[i]) + l * L * kr;
      f.y = reinterpret_cast<double*>(w + lo.y[i]) + l * nv * kr;
      f.s = static_cast<float*>(x.s) + l * x.k;
      f.other = Other + l * nv * x.k;
      f.fo = Fo + l * L * x.k;
      f.ys = reinterpret_cast<float*>(w + lo.ys[i]) + l * nv * x.k;
      f.n1 = (int)x.n1;
      f.n2 = (int)x.n2;
      f.kr = (int)kr;
      f.kout = (int)x.k;
      fin.push_back(f);
    }
  }
  // the facewise products: one descriptor per product instance, one entry
  // per 128 x 128 output tile, deepest products first (the longest tiles
  // start first)
  std::vector<pq::GemmDesc> descs;
  std::vector<pq::GemmTile> tiles;
  for (int i = 0; i < count; ++i) {
    const pq_instance& x = inst[i];
    if (!x.B) continue;
    pq::GemmDesc d;
    d.A = reinterpret_cast<const float*>(w + lo.ah[i]);
    d.B = reinterpret_cast<const float*>(w + lo.bh[i]);
    d.C = reinterpret_cast<float*>(w + lo.ch[i]);
    d.M = (int)x.n1;
    d.N = (int)x.n4;
    d.K = (int)x.n2;
    d.lda = x.n1;
    d.sA = x.n1 * x.n2;
    d.ldb = x.n2;
    d.sB = x.n2 * x.n4;
    d.ldc = x.n1;
    d.sC = x.n1 * x.n4;
    d.vec4 = pq::gemm_vec4_ok(d) ? 1 : 0;
    const int id = (int)descs.size();
    descs.push_back(d);
    for (int z = 0; z < (int)x.p; ++z)
      for (int ty = 0; ty < (d.N + 127) / 128; ++ty)
        for (int tx = 0; tx < (d.M + 127) / 128; ++tx) tiles.push_back(pq::GemmTile{id, tx, ty, z});
  }
  std::stable_sort(tiles.begin(), tiles.end(),
                   [&](const pq::GemmTile& a, const pq::GemmTile& b) { return descs[a.desc].K > descs[b.desc].K; });
  // the transforms: forward ones of every A and B, return ones of every C;
  // tiles grouped by vector width, longest tubes (most slices) first
  std::vector<pq::XformDesc> xds;
  std::vector<pq::XformTile> hts[3], uts[3];
  size_t uq[3] = {0, 0, 0};
  auto add_hat = [&](const void* in, void* out, int64_t N, const pq_instance& x) {
    const pq::XformDesc d{static_cast<const float*>(in), static_cast<const float*>(x.Q), static_cast<float*>(out), N,
                          (int)x.n3, (int)x.p};
    const int hv = pq::xform_group_vec(d);
    pq::hat_group_tiles(d, (int)xds.size(), hts[hv == 4 ? 0 : hv == 2 ? 1 : 2]);
    xds.push_back(d);
  };
  for (int i = 0; i < count; ++i) {
    const pq_instance& x = inst[i];
    add_hat(x.A, w + lo.ah[i], x.n1 * x.n2, x);
    if (x.B) add_hat(x.B, w + lo.bh[i], x.n2 * x.n4, x);
  }
  for (int i = 0; i < count; ++i) {
    const pq_instance& x = inst[i];
    if (!x.B || x.p > 32) continue;
    const pq::XformDesc d{reinterpret_cast<const float*>(w + lo.ch[i]), static_cast<const float*>(x.Q),
                          static_cast<float*>(x.C), x.n1 * x.n4, (int)x.n3, (int)x.p};
    const int uv = pq::unhat_group_vec(d);
    const int gi = uv == 4 ? 0 : uv == 2 ? 1 : 2;
    pq::unhat_group_tiles(d, (int)xds.size(), uts[gi]);
    uq[gi] = std::max(uq[gi], pq::unhat_group_q_bytes(d));
    xds.push_back(d);
  }
  XformPlan xp;
  for (int v = 0; v < 3; ++v) xp.uq[v] = uq[v];
  std::vector<pq::XformTile> htab, utab;
  auto by_n3 = [&](const pq::XformTile& a, const pq::XformTile& b) { return xds[a.desc].n3 > xds[b.desc].n3; };
  for (int v = 0; v < 3; ++v) {
    std::stable_sort(hts[v].begin(), hts[v].end(), by_n3);
    xp.nh[v] = (int)hts[v].size();
    htab.insert(htab.end(), hts[v].begin(), hts[v].end());
  }
  for (int v = 0; v < 3; ++v) {
    std::stable_sort(uts[v].begin(), uts[v].end(), by_n3);
    xp.nu[v] = (int)uts[v].size();
    utab.insert(utab.end(), uts[v].begin(), uts[v].end());
  }
  if ((int64_t)htab.size() > lo.hmax || (int64_t)utab.size() > lo.umax || (int)xds.size() > lo.nxdesc)
    return PQ_ERR_ARG;  // cannot happen: the layout counts the most tiles
  BQ_TRY(hipStreamSynchronize(stream));
  if (!lo.tab.empty())
    BQ_TRY(hipMemcpy(w + lo.faces, lo.tab.data(), sizeof(pq::JFace) * lo.tab.size(), hipMemcpyHostToDevice));
  if (lo.listed && !lo.v32.empty())
    BQ_TRY(hipMemcpy(w + lo.dv32, lo.v32.data(), sizeof(int) * lo.v32.size(), hipMemcpyHostToDevice));
  if (lo.listed && !lo.v64.empty())
    BQ_TRY(hipMemcpy(w + lo.dv64, lo.v64.data(), sizeof(int) * lo.v64.size(), hipMemcpyHostToDevice));
  for (int k = 0; k < pq::kSweepParts; ++k) {
    if (lo.listed && !lo.v32p[k].empty())
      BQ_TRY(hipMemcpy(w + lo.dv32p[k], lo.v32p[k].data(), sizeof(int) * lo.v32p[k].size(), hipMemcpyHostToDevice));
    if (lo.listed && !lo.v64p[k].empty())
      BQ_TRY(hipMemcpy(w + lo.dv64p[k], lo.v64p[k].data(), sizeof(int) * lo.v64p[k].size(), hipMemcpyHostToDevice));
  }
  if (!descs.empty())
    BQ_TRY(hipMemcpy(w + lo.gdesc, descs.data(), sizeof(pq::GemmDesc) * descs.size(), hipMemcpyHostToDevice));
  if (!tiles.empty())
    BQ_TRY(hipMemcpy(w + lo.gtile, tiles.data(), sizeof(pq::GemmTile) * tiles.size(), hipMemcpyHostToDevice));
  if (!fin.empty())
    BQ_TRY(hipMemcpy(w + lo.fin, fin.data(), sizeof(pq::FinFace) * fin.size(), hipMemcpyHostToDevice));
  if (!xds.empty())
    BQ_TRY(hipMemcpy(w + lo.xdesc, xds.data(), sizeof(pq::XformDesc) * xds.size(), hipMemcpyHostToDevice));
  if (!htab.empty())
    BQ_TRY(hipMemcpy(w + lo.htile, htab.data(), sizeof(pq::XformTile) * htab.size(), hipMemcpyHostToDevice));
  if (!utab.empty())
    BQ_TRY(hipMemcpy(w + lo.utile, utab.data(), sizeof(pq::XformTile) * utab.size(), hipMemcpyHostToDevice));
  // the second stream and the fork/join events of the float32 sweeps (the
  // captured graph keeps only the dependencies they express)
  pq::SweepPair pair;
  auto release_pair = [&]() {
    if (pair.fork) hipEventDestroy(pair.fork);
    for (int k = 0; k + 1 < pq::kSweepParts; ++k) {
      if (pair.join[k]) hipEventDestroy(pair.join[k]);
      if (pair.s2[k]) hipStreamDestroy(pair.s2[k]);
    }
  };
  hipError_t pe = hipEventCreateWithFlags(&pair.fork, hipEventDisableTiming);
  for (int k = 0; k + 1 < pq::kSweepParts && pe == hipSuccess; ++k) {
    pe = hipStreamCreateWithFlags(&pair.s2[k], hipStreamNonBlocking);
    if (pe == hipSuccess) pe = hipEventCreateWithFlags(&pair.join[k], hipEventDisableTiming);
  }
  if (pe != hipSuccess) {
    release_pair();
    return hip_rc(pe);
  }
  // one eager pass (valid outputs; tunes new launch shapes while tuning is on)
  int erc0 = enqueue(lo, inst, count, max_sweeps, tol, info_dev, w, xp, stream, &pair);
  if (erc0 == PQ_OK) erc0 = hip_rc(hipStreamSynchronize(stream));
  if (erc0 != PQ_OK) {
    release_pair();
    return erc0;
  }
  // capture the same launches on a private stream
  hipStream_t cs = nullptr;
  if ((pe = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking)) != hipSuccess) {
    release_pair();
    return hip_rc(pe);
  }
  pq_batch_s* b = new (std::nothrow) pq_batch_s;
  if (!b) {
    hipStreamDestroy(cs);
    release_pair();
    return PQ_ERR_ARG;
  }
  int rc = hip_rc(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
  if (rc == PQ_OK) {
    const int erc = enqueue(lo, inst, count, max_sweeps, tol, info_dev, w, xp, cs, &pair);
    hipGraph_t g = nullptr;
    const int crc = hip_rc(hipStreamEndCapture(cs, &g));
    rc = erc != PQ_OK ? erc : crc;
    b->graph = g;
    if (rc == PQ_OK) rc = hip_rc(hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0));
  }
  hipStreamDestroy(cs);
  release_pair();
  if (rc != PQ_OK) {
    if (b->exec) hipGraphExecDestroy(b->exec);
    if (b->graph) hipGraphDestroy(b->graph);
    delete b;
    return rc;
  }
  *out = b;
  return PQ_OK;
}

int pq_batched_run(pq_batch batch, hipStream_t stream) {
  if (!batch || !batch->exec) return PQ_ERR_NULL;
  return hip_rc(hipGraphLaunch(batch->exec, stream));
}

int pq_batched_destroy(pq_batch batch) {
  if (!batch) return PQ_ERR_NULL;
  if (batch->exec) hipGraphExecDestroy(batch->exec);
  if (batch->graph) hipGraphDestroy(batch->graph);
  delete batch;
  return PQ_OK;
}

}  // extern "C"
