// C ABI of libppl: planner, workspace binding, build / contract / iterate drivers.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <new>

#include "diis_solve.h"
#include "pack_cubes.h"
#include "ppl_internal.h"

// Resident upper-triangle builds write the GEMM's natural layout and pack whole V+- rows,
// mirror entries included, in one pass (0: G blocks, packing of the upper triangle, then a
// separate mirror pass, as streaming steps still do).
#ifndef PPL_PACK_CUBES
#define PPL_PACK_CUBES 1
#endif
constexpr bool kPackCubes = PPL_PACK_CUBES;

namespace ppl {

static thread_local char g_err[1024] = "";

void set_error(const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof(g_err), fmt, ap);
  va_end(ap);
}

int fail(int code, const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof(g_err), fmt, ap);
  va_end(ap);
  return code;
}

static uint64_t align256(uint64_t x) { return (x + 255) / 256 * 256; }

// bytes per element of an operand plane and number of planes
static int elem_bytes(int prec) { return prec == PPL_FP64 ? 8 : (prec == PPL_FP32 ? 4 : 2); }
static int planes(int prec) { return prec == PPL_BF16X3 ? 2 : (prec == PPL_BF16X6 ? 3 : 1); }
static int acc_bytes(int prec) { return prec == PPL_FP64 ? 8 : 4; }

// overflow-checked multiply of non-negative sizes
static bool mul_ok(uint64_t a, uint64_t b, uint64_t* out) {
  if (a != 0 && b > UINT64_MAX / a) return false;
  *out = a * b;
  return true;
}

struct Layout {
  uint64_t cur = 0;
  Region take(uint64_t bytes) {
    Region r;
    r.off = cur;
    r.bytes = align256(bytes);
    cur += r.bytes;
    return r;
  }
};

// Scratch of the ring terms: staged Cholesky blocks (ov, oo, vv rows of P), the (kj|bc)
// product, and seven (o v) x (o v) pair matrices. With lp_prec (a plan whose low-precision
// sweeps run the ring GEMMs in that precision) also J and K in it, jl and kl: one region
// each of its planes back to back (FP32: one; BF16x3: hi, lo; BF16x6: hi, mid, lo).
struct RingLayout {
  int64_t ldx = 0, ldk = 0, ldg = 0;
  uint64_t xov = 0, xoo = 0, xvv = 0, g = 0, j = 0, k = 0, xa = 0, an = 0, b = 0, c1 = 0, c2 = 0, bytes = 0;
  int lp_prec = PPL_FP64;
  uint64_t jl = 0, kl = 0, lp_plane = 0;   // low-precision J, K and the bytes of one of their planes
};

static bool ring_layout(int64_t o, int64_t v, int64_t naux, RingLayout& r, int lp_prec = PPL_FP64) {
  if (o < 1 || v < 1 || naux < 1 || o > 32767 || v > 32767) return false;
  r.ldx = pad_ld(naux);
  r.ldk = pad_ld(o * v);
  r.ldg = pad_ld(v * v);
  uint64_t x;
  if (!mul_ok((uint64_t)(o * v), (uint64_t)r.ldk, &x) || !mul_ok(x, 16, &x)) return false;
  if (!mul_ok((uint64_t)(v * v), (uint64_t)r.ldx, &x) || !mul_ok(x, 16, &x)) return false;
  // the regions together (below) must not overflow 64-bit byte counts either
  const double total = 8.0 * ((double)(o * v + o * o + v * v) * (double)r.ldx + (double)(o * o) * (double)r.ldg +
                              9.0 * (double)(o * v) * (double)r.ldk) + 12.0 * (double)(o * v) * (double)r.ldk;
  if (total > 4.0e18) return false;
  Layout L;
  r.xov = L.take((uint64_t)o * v * r.ldx * 8).off;
  r.xoo = L.take((uint64_t)o * o * r.ldx * 8).off;
  r.xvv = L.take((uint64_t)v * v * r.ldx * 8).off;
  r.g = L.take((uint64_t)o * o * r.ldg * 8).off;
  const uint64_t m = (uint64_t)o * v * r.ldk * 8;
  r.j = L.take(m).off;
  r.k = L.take(m).off;
  r.xa = L.take(m).off;
  r.an = L.take(m).off;
  r.b = L.take(m).off;
  r.c1 = L.take(m).off;
  r.c2 = L.take(m).off;
  r.lp_prec = lp_prec;
  if (lp_prec != PPL_FP64) {
    r.lp_plane = (uint64_t)o * v * r.ldk * elem_bytes(lp_prec);
    r.jl = L.take(r.lp_plane * planes(lp_prec)).off;
    r.kl = L.take(r.lp_plane * planes(lp_prec)).off;
  }
  r.bytes = L.cur;
  return true;
}

// Split virtual rows a into build steps whose pair count (sum of v - a) stays
// within cap (at least one row per step).
static void make_batches(int v, int64_t cap, std::vector<Batch>& out) {
  out.clear();
  int a = 0;
  while (a < v) {
    int a1 = a;
    int64_t pairs = 0;
    while (a1 < v && (a1 == a || pairs + (v - a1) <= cap)) {
      pairs += v - a1;
      ++a1;
    }
    Batch b;
    b.a0 = a;
    b.a1 = a1;
    b.p0 = pair_plus(a, a, v);
    b.p1 = (a1 >= v) ? npairs_plus(v) : pair_plus(a1, a1, v);
    b.q0 = (a < v - 1) ? pair_minus(a, a + 1, v) : npairs_minus(v);
    b.q1 = (a1 >= v - 1) ? npairs_minus(v) : pair_minus(a1, a1 + 1, v);
    if (b.q1 < b.q0) b.q1 = b.q0;
    out.push_back(b);
    a = a1;
  }
}

// Bytes per element of the build scratch G: the widest accumulator among the
// operand sets the plan builds (a mixed plan with an FP64 copy needs 8).
static int g_acc_bytes(ppl_plan_t p) {
  int w = 0;
  for (int k = 0; k < 2; ++k)
    if (p->ops[k].present) w = std::max(w, acc_bytes(p->ops[k].prec));
  return w;
}

// Tuned contraction configurations: "ppl-tune 1 prec o v tile+ splits+ tile- splits-" per
// line; the last line matching (prec, o, v) wins. Unreadable files and foreign lines are
// skipped, and so are BF16x6 lines whose K decomposition breaks the slice-length rule of
// that precision (stream-K, or fewer slices than contract_min_splits for the padded K of
// R+ (ldp) or R- (ldm)): the file is user-editable text and must not loosen accuracy.
static bool tune_cache_lookup(const std::string& path, int prec, int o, int v, int64_t ldp, int64_t ldm,
                              int cfg[4]) {
  if (path.empty()) return false;
  FILE* f = fopen(path.c_str(), "r");
  if (!f) return false;
  char line[256];
  bool found = false;
  while (fgets(line, sizeof(line), f)) {
    int ver, pr, oo, vv, c[4];
    if (sscanf(line, "ppl-tune %d %d %d %d %d %d %d %d", &ver, &pr, &oo, &vv, &c[0], &c[1], &c[2], &c[3]) != 8)
      continue;
    if (ver != 1 || pr != prec || oo != o || vv != v) continue;
    if (c[0] < 0 || c[0] >= contract_tile_count() || c[2] < 0 || c[2] >= contract_tile_count()) continue;
    if (c[1] < 0 || c[1] > kMaxSplits || c[3] < 0 || c[3] > kMaxSplits) continue;
    if (prec == PPL_BF16X6 && (c[1] == 0 || c[1] < contract_min_splits(prec, ldp) || c[3] == 0 ||
                               c[3] < contract_min_splits(prec, ldm)))
      continue;
    for (int k = 0; k < 4; ++k) cfg[k] = c[k];
    found = true;
  }
  fclose(f);
  return found;
}

static int tune_cache_append(const std::string& path, int prec, int o, int v, const int cfg[4]) {
  FILE* f = fopen(path.c_str(), "a");
  if (!f) return fail(PPL_E_ARG, "cannot write the tune cache %s", path.c_str());
  const int n = fprintf(f, "ppl-tune 1 %d %d %d %d %d %d %d\n", prec, o, v, cfg[0], cfg[1], cfg[2], cfg[3]);
  const int c = fclose(f);
  if (n < 0 || c != 0) return fail(PPL_E_ARG, "cannot write the tune cache %s", path.c_str());
  return PPL_OK;
}

// Scratch of the hole-hole ladder, carved from the build scratch G: staged occupied
// block, (ki|lj), W+- [N+][ldq] / [N-][ldqm], and one chunk of virtual-pair rows of the
// transposed amplitudes and of the transposed results ([chunk][ldq] each; ldq >= ldqm).
// The floor (avail == 0) takes chunks of at most kHhlChunk rows; given the scratch
// actually available, chunks grow to use it.
constexpr int64_t kHhlChunk = 8192;
struct HhlScratch {
  int64_t ldq, ldqm, chunk;
  uint64_t xoo, woo, wp, wm, st, cp, bytes;
};
static HhlScratch hhl_scratch(ppl_plan_t p, uint64_t avail = 0) {
  HhlScratch h{};
  const int64_t o = p->o, Nmq = std::max<int64_t>(p->Nm, 1);
  h.ldq = pad_ld(p->Np);
  h.ldqm = pad_ld(Nmq);
  uint64_t cur = 0;
  auto take = [&](uint64_t b) {
    const uint64_t at = cur;
    cur = align256(cur + b);
    return at;
  };
  h.xoo = take((uint64_t)o * o * p->ldx * 8);
  h.woo = take((uint64_t)o * o * o * o * 8);
  h.wp = take((uint64_t)p->Np * h.ldq * 8);
  h.wm = take((uint64_t)Nmq * h.ldqm * 8);
  const uint64_t row = (uint64_t)h.ldq * 8;
  h.chunk = std::min<int64_t>(p->Pp, kHhlChunk);
  if (avail > cur + 2 * (uint64_t)h.chunk * row + 1024)
    h.chunk = std::min<int64_t>(p->Pp, (int64_t)((avail - cur - 1024) / (2 * row)));
  h.st = take((uint64_t)h.chunk * row);
  h.cp = take((uint64_t)h.chunk * row);
  h.bytes = cur;
  return h;
}

// Assign every workspace region for a given G cap and residency; returns total bytes.
static uint64_t assign_layout(ppl_plan_t p, int64_t gcap, bool resident, int64_t max_batch_pairs) {
  Layout L;
  const int64_t v = p->v, o = p->o;
  for (int k = 0; k < 2; ++k) {
    OperandSet& s = p->ops[k];
    if (!s.present) continue;
    const uint64_t w = elem_bytes(s.prec);
    const int np = planes(s.prec);
    const int64_t vrows_p = resident ? p->Pp : max_batch_pairs;
    const int64_t vrows_m = resident ? p->Pm : max_batch_pairs;
    if (np == 3) {
      // BF16x6: the mid and lo planes follow their hi plane directly (three planes spaced
      // one plane apart; the kernels find lo at mid + (mid - hi))
      auto three = [&](Region& hi, Region& rest, uint64_t bytes) {
        hi = L.take(bytes);
        rest = L.take(2 * hi.bytes);
      };
      three(s.xt, s.xt_lo, (uint64_t)v * v * p->ldx * w);
      three(s.vp, s.vp_lo, (uint64_t)vrows_p * p->ldp * w);
      three(s.vm, s.vm_lo, (uint64_t)std::max<int64_t>(vrows_m, 1) * p->ldm * w);
      three(s.sp, s.sp_lo, (uint64_t)p->Np * p->ldp * w);
      three(s.am, s.am_lo, (uint64_t)std::max<int64_t>(p->Nm, 1) * p->ldm * w);
      continue;
    }
    s.xt = L.take((uint64_t)v * v * p->ldx * w);
    s.vp = L.take((uint64_t)vrows_p * p->ldp * w);
    s.vm = L.take((uint64_t)std::max<int64_t>(vrows_m, 1) * p->ldm * w);
    s.sp = L.take((uint64_t)p->Np * p->ldp * w);
    s.am = L.take((uint64_t)std::max<int64_t>(p->Nm, 1) * p->ldm * w);
    if (np == 2) {
      s.xt_lo = L.take(s.xt.bytes);
      s.vp_lo = L.take(s.vp.bytes);
      s.vm_lo = L.take(s.vm.bytes);
      s.sp_lo = L.take(s.sp.bytes);
      s.am_lo = L.take(s.am.bytes);
    } else {
      s.xt_lo = s.vp_lo = s.vm_lo = s.sp_lo = s.am_lo = Region{};
    }
  }
  // build scratch G (accumulator precision) doubles as the (ia|jb) scratch
  // (the (ia|jb) scratch of the iteration only when the plan iterates)
  const uint64_t gbytes = std::max<uint64_t>(std::max<uint64_t>((uint64_t)gcap * v * v * g_acc_bytes(p),
                                                               p->contract_only ? 0 : (uint64_t)(o * v) * (o * v) * 8),
                                             hhl_scratch(p).bytes);
  p->g_bytes_wanted = align256(gbytes);
  p->g = L.take(p->g_external ? 0 : gbytes);
  if (p->ring) {
    RingLayout rl;
    ring_layout(p->o, p->v, p->naux, rl, p->ops[0].prec);
    p->ring_ws = L.take(rl.bytes);
    p->tfull = L.take((uint64_t)o * o * v * v * 8);
    p->rfull = L.take((uint64_t)o * o * v * v * 8);
  } else {
    p->ring_ws = p->tfull = p->rfull = Region{};
  }
  p->rp = L.take((uint64_t)p->Np * p->ldp * 8);
  p->rm = L.take((uint64_t)std::max<int64_t>(p->Nm, 1) * p->ldm * 8);
  // split-K slices for up to kMaxSplits (autotuning may pick any count), sized for FP64,
  // or the stream-K partial slots of the largest tile, whichever is larger. A resident
  // plan's slices span all columns; a streaming plan's span the widest batch only.
  p->ld_part = resident ? std::max(p->ldp, p->ldm) : pad_ld(std::max<int64_t>(max_batch_pairs, 1));
  uint64_t part_bytes = (uint64_t)std::max(p->Np, p->Nm) * p->ld_part * kMaxSplits * 8;
  for (int t = 0; t < contract_tile_count(); ++t) {
    part_bytes = std::max(part_bytes, streamk_part_bytes(t, PPL_FP64, p->Np, resident ? p->Pp : max_batch_pairs, p->ldp));
    if (p->Nm > 0)
      part_bytes = std::max(part_bytes, streamk_part_bytes(t, PPL_FP64, p->Nm, resident ? p->Pm : max_batch_pairs, p->ldm));
  }
  p->part = L.take(part_bytes);
  if (p->ops[0].prec != PPL_FP64) {   // FP64 master amplitudes
    p->s64 = L.take((uint64_t)p->Np * p->ldp * 8);
    p->a64 = L.take((uint64_t)std::max<int64_t>(p->Nm, 1) * p->ldm * 8);
  } else {
    p->s64 = p->ops[0].sp;
    p->a64 = p->ops[0].am;
  }
  if (p->contract_only) {
    p->bs = p->ba = p->vs = p->va = p->xov = Region{};
  } else {
    p->bs = L.take((uint64_t)p->Np * p->ldp * 8);     // backup of S'/A' for checked starts
    p->ba = L.take((uint64_t)std::max<int64_t>(p->Nm, 1) * p->ldm * 8);
    p->vs = L.take((uint64_t)p->Np * p->ldp * 8);
    p->va = L.take((uint64_t)std::max<int64_t>(p->Nm, 1) * p->ldm * 8);
    p->xov = L.take((uint64_t)o * v * p->ldx * 8);
  }
  p->tab_vp = L.take((uint64_t)p->Pp * 4);
  p->tab_vm = L.take((uint64_t)std::max<int64_t>(p->Pm, 1) * 4);
  p->tab_op = L.take((uint64_t)p->Np * 4);
  p->tab_om = L.take((uint64_t)std::max<int64_t>(p->Nm, 1) * 4);
  p->red = L.take((uint64_t)(kReduceBlocks * 4 + 8) * 8);
  p->diis_slot_n = p->Np * p->ldp + std::max<int64_t>(p->Nm, 1) * p->ldm;
  if (p->diis_max > 0) {
    p->diis_t = L.take((uint64_t)p->diis_max * p->diis_slot_n * 8);
    p->diis_e = L.take((uint64_t)p->diis_max * p->diis_slot_n * 8);
    p->diis_red = L.take((uint64_t)(kReduceBlocks + 1) * kDiisMax * 8);
  } else {
    p->diis_t = p->diis_e = p->diis_red = Region{};
  }
  p->tiles = L.take((uint64_t)p->tiles_host.size() * 4);
  p->cols = p->sym_build ? L.take((uint64_t)npairs_plus(v) * 4) : Region{};
  p->cube_off = (p->sym_build && resident && kPackCubes) ? L.take((uint64_t)(v + 1) * 8) : Region{};
  p->r2p = p->r2m = p->ut = Region{};
  if (p->sym_build && !resident) {
    // the K range of a step starts at its first pair rounded down to 64, so it spans at
    // most the step's pairs plus 63
    p->ldq = pad_ld(p->Np);
    p->ldqm = pad_ld(std::max<int64_t>(p->Nm, 1));
    p->ldk = pad_ld(max_batch_pairs + 63);
    p->r2p = L.take((uint64_t)p->Pp * p->ldq * 8);
    p->r2m = L.take((uint64_t)std::max<int64_t>(p->Pm, 1) * p->ldqm * 8);
    p->ut = L.take((uint64_t)p->Pp * p->ldk * 8);
  }
  return L.cur;
}

// Build tile lists per step: set 0 for the plan's operands, set 1 for the FP64 copy of
// a mixed plan when that builds on another tile.
static void make_tile_tables(ppl_plan_t p) {
  p->tiles_host.clear();
  p->tiles_off.clear();
  p->tiles_n.clear();
  p->tile_sets = (p->ops[1].present && p->tile_build64 != p->tile_build) ? 2 : 1;
  for (int set = 0; set < p->tile_sets; ++set) {
    const int tile = set ? p->tile_build64 : p->tile_build;
    for (const Batch& b : p->batches) {
      std::vector<int> list;
      int nmt, nnt;
      if (p->sym_build) build_tile_table_sym(tile, p->v, b.a0, b.a1, list, nmt, nnt);
      else build_tile_table(tile, p->v, b.a0, b.a1, list, nmt, nnt);
      p->tiles_off.push_back((int64_t)p->tiles_host.size());
      p->tiles_n.push_back((int64_t)list.size() / 2);
      p->tiles_host.insert(p->tiles_host.end(), list.begin(), list.end());
    }
  }
}

int autotune_impl(ppl_plan_t p, int32_t reps, double* best_ms);

static int check_plan(ppl_plan_t p) {
  if (!p) return fail(PPL_E_ARG, "null plan");
  return PPL_OK;
}

static int check_bound(ppl_plan_t p) {
  PPL_TRY(check_plan(p));
  if (!p->ws) return fail(PPL_E_STATE, "no workspace bound (call ppl_bind_workspace first)");
  return PPL_OK;
}

// ---------------------------------------------------------------- launch timing
// Scoped pair of events around one or more launches of one kind.
struct ProfScope {
  ppl_plan_t p;
  int idx = -1;
  ProfScope(ppl_plan_t plan, int kind, double flops) : p(plan) {
    if (!p->prof_on) return;
    if (p->prof_next + 2 > (int)p->prof_pool.size()) {
      for (int k = 0; k < 64; ++k) {
        hipEvent_t e;
        if (hipEventCreate(&e) != hipSuccess) return;
        p->prof_pool.push_back(e);
      }
    }
    idx = p->prof_next;
    p->prof_next += 2;
    if (hipEventRecord(p->prof_pool[idx], p->stream) != hipSuccess) { idx = -1; return; }
    p->prof_recs.push_back({kind, idx, flops});
  }
  ~ProfScope() {
    if (idx >= 0) (void)hipEventRecord(p->prof_pool[idx + 1], p->stream);
  }
};


// ------------------------------------------------------------------ build
// Useful flops of building virtual rows a in [a0, a1): 2 naux v^2 per pair (a <= b) for full
// rows; 2 naux (v - a)^2 (v - a + 1) / 2 per virtual a for the upper triangle (rows
// (a, c >= a), columns the packed pairs (b <= d) with b >= a).
static double build_flops(ppl_plan_t p, int a0, int a1) {
  double f = 0.0;
  for (int a = a0; a < a1; ++a) {
    const double w = (double)(p->v - a);
    f += p->sym_build ? w * w * (w + 1.0) / 2.0 : (double)p->v * p->v * w;
  }
  return 2.0 * p->naux * f;
}

static int mirror_vpm(ppl_plan_t p, OperandSet& s) {
  if (!p->sym_build || kPackCubes) return PPL_OK;   // the cube packing writes the mirror entries itself
  ProfScope ps(p, PPL_PROF_BUILD_PACK, 0.0);
  const int w = elem_bytes(s.prec);
  const int np = planes(s.prec);
  // plane k of a region starts k plane sizes after its hi plane (the lo planes of BF16x6
  // follow the hi plane directly; the lo plane of BF16x3 lies elsewhere)
  for (int k = 0; k < np; ++k) {
    char* vp = k == 0 ? at<char>(p, s.vp) : at<char>(p, s.vp_lo) + (uint64_t)(k - 1) * s.vp.bytes;
    PPL_TRY(mirror_lower(p->stream, w, vp, p->Pp, p->ldp));
    if (p->Pm > 0) {
      char* vm = k == 0 ? at<char>(p, s.vm) : at<char>(p, s.vm_lo) + (uint64_t)(k - 1) * s.vm.bytes;
      PPL_TRY(mirror_lower(p->stream, w, vm, p->Pm, p->ldm));
    }
  }
  return PPL_OK;
}

static int build_one(ppl_plan_t p, OperandSet& s, const double* L, int bi, bool staged) {
  const Batch& b = p->batches[bi];
  hipStream_t st = p->stream;
  if (!staged) {
    ProfScope ps(p, PPL_PROF_OTHER, 0.0);
    PPL_TRY(stage_vv(st, s.prec, L, p->o, p->v, p->naux, p->ldx, at<void>(p, s.xt),
                     s.xt_lo.bytes ? at<void>(p, s.xt_lo) : nullptr));
  }
  // the FP64 copy of a mixed plan builds on the FP64 build tile, with its own lists
  const int set = (&s == &p->ops[1] && p->tile_sets == 2) ? 1 : 0;
  const int tile = (&s == &p->ops[1]) ? p->tile_build64 : p->tile_build;
  const size_t ti = (size_t)set * p->batches.size() + (size_t)bi;
  const int* dtiles = at<int>(p, p->tiles) + p->tiles_off[ti];
  const int64_t nvalid = p->tiles_n[ti];
  // every write of this step must stay inside its region
  const uint64_t g_need = (uint64_t)(b.p1 - b.p0) * p->v * p->v * acc_bytes(s.prec);
  if (g_need > p->g.bytes)
    return fail(PPL_E_STATE, "build step %d needs %llu B of scratch, plan has %llu B", bi,
                (unsigned long long)g_need, (unsigned long long)p->g.bytes);
  {
    const int64_t r0p = p->resident ? b.p0 : 0, r0m = p->resident ? b.q0 : 0;
    const uint64_t w = (uint64_t)elem_bytes(s.prec);
    if ((uint64_t)(r0p + (b.p1 - b.p0)) * p->ldp * w > s.vp.bytes ||
        (uint64_t)(r0m + (b.q1 - b.q0)) * p->ldm * w > s.vm.bytes)
      return fail(PPL_E_STATE, "build step %d exceeds the V+- rows of the plan", bi);
  }
  if (p->sym_build && p->resident && kPackCubes) {
    // natural GEMM layout, then whole rows and their mirror entries in one packing pass
    {
      ProfScope ps(p, PPL_PROF_BUILD_GEMM, build_flops(p, b.a0, b.a1));
      PPL_TRY(gemm_build_natural(st, s.prec, tile, p->v, b.a0, b.a1, p->ldx, at<void>(p, s.xt),
                                 s.xt_lo.bytes ? at<void>(p, s.xt_lo) : nullptr, p->ldx, at<void>(p, p->g), dtiles,
                                 nvalid, at<int>(p, p->tab_vp), at<int>(p, p->cols)));
    }
    ProfScope ps(p, PPL_PROF_BUILD_PACK, 0.0);
    const int64_t W = p->v - b.a0;
    return pack_vpm_cubes(st, s.prec, p->v, b.a0, b.a1, at<void>(p, p->g), W * (W + 1) / 2,
                          at<int64_t>(p, p->cube_off), at<void>(p, s.vp), s.vp_lo.bytes ? at<void>(p, s.vp_lo) : nullptr,
                          p->ldp, at<void>(p, s.vm), s.vm_lo.bytes ? at<void>(p, s.vm_lo) : nullptr, p->ldm);
  }
  if (p->sym_build) {
    {
      ProfScope ps(p, PPL_PROF_BUILD_GEMM, build_flops(p, b.a0, b.a1));
      PPL_TRY(gemm_build_sym(st, s.prec, tile, p->v, b.a0, b.a1, p->ldx, at<void>(p, s.xt),
                             s.xt_lo.bytes ? at<void>(p, s.xt_lo) : nullptr, p->ldx, at<void>(p, p->g), dtiles,
                             nvalid, at<int>(p, p->tab_vp), at<int>(p, p->cols)));
    }
    ProfScope ps(p, PPL_PROF_BUILD_PACK, 0.0);
    const bool str = !p->resident;
    return pack_vpm_sym(st, s.prec, p->v, b.a0, b.a1, at<void>(p, p->g), at<void>(p, s.vp),
                        s.vp_lo.bytes ? at<void>(p, s.vp_lo) : nullptr, p->ldp, at<void>(p, s.vm),
                        s.vm_lo.bytes ? at<void>(p, s.vm_lo) : nullptr, p->ldm, at<int>(p, p->tab_vp),
                        str ? b.p0 : 0, str ? b.q0 : 0, str ? 1 : 0, b.p0 / 64 * 64, b.q0 / 64 * 64);
  }
  {
    ProfScope ps(p, PPL_PROF_BUILD_GEMM, build_flops(p, b.a0, b.a1));
    PPL_TRY(gemm_build(st, s.prec, tile, p->v, b.a0, b.a1, p->ldx, at<void>(p, s.xt),
                       s.xt_lo.bytes ? at<void>(p, s.xt_lo) : nullptr, p->ldx, at<void>(p, p->g), dtiles,
                       nvalid));
  }
  const int64_t row0p = p->resident ? 0 : b.p0;
  const int64_t row0m = p->resident ? 0 : b.q0;
  ProfScope ps(p, PPL_PROF_BUILD_PACK, 0.0);
  PPL_TRY(pack_vpm(st, s.prec, p->v, b.a0, b.a1, at<void>(p, p->g), at<void>(p, s.vp),
                   s.vp_lo.bytes ? at<void>(p, s.vp_lo) : nullptr, p->ldp, row0p, at<void>(p, s.vm),
                   s.vm_lo.bytes ? at<void>(p, s.vm_lo) : nullptr, p->ldm, row0m,
                   at<int>(p, p->tab_vp), at<int>(p, p->tab_vm)));
  return PPL_OK;
}

static int build_all(ppl_plan_t p, OperandSet& s, const double* L) {
  for (int bi = 0; bi < (int)p->batches.size(); ++bi) PPL_TRY(build_one(p, s, L, bi, bi > 0));
  PPL_TRY(mirror_vpm(p, s));
  s.built = true;
  return PPL_OK;
}

// ------------------------------------------------------------------ contraction of packed operands
// Streaming with upper-triangle steps (FP64): V = U + U^T, U the rows of a step from their
// own pair on, diagonal halved. Per step, R[:, step] = S' U_step^T over K from the step's
// first pair (rounded down to 64; U is zero before its own pair there), and
// R^T[k0:, :] += U_step^T S'[:, step]^T with the step's pairs as K, through a transposed
// copy of the step's rows. The transposed sums are added into R+- after the last step.
static int contract_stream_sym(ppl_plan_t p, OperandSet& s, int tile, int tile_m, int split_p, int split_m,
                               void* part) {
  hipStream_t st = p->stream;
  if (s.prec != PPL_FP64 || !p->r2p.bytes || !p->ut.bytes)
    return fail(PPL_E_STATE, "streaming upper-triangle plan without its buffers");
  double* sp = at<double>(p, s.sp);
  double* am = at<double>(p, s.am);
  double* vp = at<double>(p, s.vp);
  double* vm = at<double>(p, s.vm);
  double* rp = at<double>(p, p->rp);
  double* rm = at<double>(p, p->rm);
  double* r2p = at<double>(p, p->r2p);
  double* r2m = at<double>(p, p->r2m);
  double* ut = at<double>(p, p->ut);
  PPL_TRY(zero_bytes(st, r2p, p->r2p.bytes));
  if (p->Nm > 0) PPL_TRY(zero_bytes(st, r2m, p->r2m.bytes));
  int t2p = -1, s2p = 1, t2m = -1, s2m = 1;
  contract_choose(PPL_FP64, p->Pp, p->Np, p->ldk, 1, &t2p, &s2p);
  if (p->Nm > 0) contract_choose(PPL_FP64, p->Pm, p->Nm, p->ldk, 1, &t2m, &s2m);
  // one half (U or U^T) of a step's rows [r0, r1) of an n-row block: useful flops
  auto half_flops = [](int64_t rows, int64_t n, int64_t r0, int64_t r1) {
    const double w = (double)(r1 - r0);
    return 2.0 * rows * (w * n - (double)(r0 + r1 - 1) * w / 2.0);
  };
  for (int bi = 0; bi < (int)p->batches.size(); ++bi) {
    const Batch& b = p->batches[bi];
    PPL_TRY(build_one(p, s, p->L_last, bi, bi > 0));
    {
      ProfScope ps(p, PPL_PROF_CONTRACT_PLUS, 2.0 * half_flops(p->Np, p->Pp, b.p0, b.p1));
      const int64_t k0 = b.p0 / 64 * 64, w = b.p1 - b.p0, K2 = pad_ld(b.p1 - k0), nr = p->Pp - k0;
      if (K2 > p->ldk) return fail(PPL_E_STATE, "step %d exceeds the transposed block", bi);
      PPL_TRY(gemm_contract(st, PPL_FP64, tile, p->Np, w, p->ldp - k0, sp + k0, nullptr, p->ldp, vp + k0, nullptr,
                            p->ldp, rp, p->ldp, b.p0, split_p, part, p->ld_part, p->part.bytes));
      PPL_TRY(transpose_block(st, 8, vp, p->ldp, b.p0, b.p1, k0, k0, ut, p->ldk, nr, K2));
      PPL_TRY(gemm_contract(st, PPL_FP64, t2p, nr, p->Np, K2, ut, nullptr, p->ldk, sp + k0, nullptr, p->ldp,
                            r2p + k0 * p->ldq, p->ldq, 0, 1, nullptr, p->ldq, 0, true));
    }
    if (p->Nm > 0 && b.q1 > b.q0) {
      ProfScope ps(p, PPL_PROF_CONTRACT_MINUS, 2.0 * half_flops(p->Nm, p->Pm, b.q0, b.q1));
      const int64_t k0 = b.q0 / 64 * 64, w = b.q1 - b.q0, K2 = pad_ld(b.q1 - k0), nr = p->Pm - k0;
      if (K2 > p->ldk) return fail(PPL_E_STATE, "step %d exceeds the transposed block", bi);
      PPL_TRY(gemm_contract(st, PPL_FP64, tile_m, p->Nm, w, p->ldm - k0, am + k0, nullptr, p->ldm, vm + k0, nullptr,
                            p->ldm, rm, p->ldm, b.q0, split_m, part, p->ld_part, p->part.bytes));
      PPL_TRY(transpose_block(st, 8, vm, p->ldm, b.q0, b.q1, k0, k0, ut, p->ldk, nr, K2));
      PPL_TRY(gemm_contract(st, PPL_FP64, t2m, nr, p->Nm, K2, ut, nullptr, p->ldk, am + k0, nullptr, p->ldm,
                            r2m + k0 * p->ldqm, p->ldqm, 0, 1, nullptr, p->ldqm, 0, true));
    }
  }
  ProfScope ps(p, PPL_PROF_OTHER, 0.0);
  PPL_TRY(add_transposed(st, PPL_FP64, rp, p->ldp, r2p, p->ldq, p->Np, p->Pp));
  if (p->Nm > 0) PPL_TRY(add_transposed(st, PPL_FP64, rm, p->ldm, r2m, p->ldqm, p->Nm, p->Pm));
  return PPL_OK;
}

// R+ = S' V+^T, R- = A' V-^T with the operand set s (its S'/A' must be current).
static int contract_packed(ppl_plan_t p, OperandSet& s) {
  hipStream_t st = p->stream;
  const void* sp = at<void>(p, s.sp);
  const void* sp_lo = s.sp_lo.bytes ? at<void>(p, s.sp_lo) : nullptr;
  const void* am = at<void>(p, s.am);
  const void* am_lo = s.am_lo.bytes ? at<void>(p, s.am_lo) : nullptr;
  const bool primary = &s == &p->ops[0];
  const int tile = primary ? p->tile_contract : s.tile_p, tile_m = primary ? p->tile_m : s.tile_m;
  const int split_p = primary ? p->split_p : s.split_p, split_m = primary ? p->split_m : s.split_m;
  void* part = p->part.bytes ? at<void>(p, p->part) : nullptr;
  if (std::max(split_p, split_m) > kMaxSplits ||
      (uint64_t)std::max(p->Np, p->Nm) * p->ld_part * kMaxSplits * 8 > p->part.bytes ||
      (uint64_t)p->Np * p->ldp * 8 > p->rp.bytes)
    return fail(PPL_E_STATE, "contraction buffers smaller than the plan requires");
  const double fp = 2.0 * (double)p->Np * p->Pp, fm = 2.0 * (double)p->Nm * p->Pm;
  if (p->resident) {
    if (!s.built) return fail(PPL_E_STATE, "V+- not built (call ppl_build_batch first)");
    {
      ProfScope ps(p, PPL_PROF_CONTRACT_PLUS, fp * p->Pp);
      PPL_TRY(gemm_contract(st, s.prec, tile, p->Np, p->Pp, p->ldp, sp, sp_lo, p->ldp,
                            at<void>(p, s.vp), s.vp_lo.bytes ? at<void>(p, s.vp_lo) : nullptr, p->ldp,
                            at<void>(p, p->rp), p->ldp, 0, split_p, part, p->ld_part, p->part.bytes));
    }
    ProfScope ps(p, PPL_PROF_CONTRACT_MINUS, fm * p->Pm);
    if (p->Nm > 0 && p->Pm > 0)
      PPL_TRY(gemm_contract(st, s.prec, tile_m, p->Nm, p->Pm, p->ldm, am, am_lo, p->ldm,
                            at<void>(p, s.vm), s.vm_lo.bytes ? at<void>(p, s.vm_lo) : nullptr, p->ldm,
                            at<void>(p, p->rm), p->ldm, 0, split_m, part, p->ld_part, p->part.bytes));
    return PPL_OK;
  }
  if (!p->L_last) return fail(PPL_E_STATE, "streaming plan has no Cholesky vectors (call ppl_build_batch)");
  if (p->sym_build) return contract_stream_sym(p, s, tile, tile_m, split_p, split_m, part);
  for (int bi = 0; bi < (int)p->batches.size(); ++bi) {
    const Batch& b = p->batches[bi];
    PPL_TRY(build_one(p, s, p->L_last, bi, bi > 0));
    {
      ProfScope ps(p, PPL_PROF_CONTRACT_PLUS, 2.0 * (double)p->Np * p->Pp * (double)(b.p1 - b.p0));
      PPL_TRY(gemm_contract(st, s.prec, tile, p->Np, b.p1 - b.p0, p->ldp, sp, sp_lo, p->ldp,
                            at<void>(p, s.vp), s.vp_lo.bytes ? at<void>(p, s.vp_lo) : nullptr, p->ldp,
                            at<void>(p, p->rp), p->ldp, b.p0, split_p, part, p->ld_part, p->part.bytes));
    }
    ProfScope ps(p, PPL_PROF_CONTRACT_MINUS, 2.0 * (double)p->Nm * p->Pm * (double)(b.q1 - b.q0));
    if (p->Nm > 0 && b.q1 > b.q0)
      PPL_TRY(gemm_contract(st, s.prec, tile_m, p->Nm, b.q1 - b.q0, p->ldm, am, am_lo, p->ldm,
                            at<void>(p, s.vm), s.vm_lo.bytes ? at<void>(p, s.vm_lo) : nullptr, p->ldm,
                            at<void>(p, p->rm), p->ldm, b.q0, split_m, part, p->ld_part, p->part.bytes));
  }
  return PPL_OK;
}

// refresh the low-precision S'/A' copies of set s from the FP64 master
static int refresh_operands(ppl_plan_t p, OperandSet& s) {
  if (s.prec == PPL_FP64) {
    if (s.sp.off != p->s64.off) {   // FP64 refinement set of a mixed plan: copy the master
      PPL_TRY(convert_rows(p->stream, PPL_FP64, at<double>(p, p->s64), p->Np, p->Pp, p->ldp,
                           at<void>(p, s.sp), nullptr));
      if (p->Nm > 0)
        PPL_TRY(convert_rows(p->stream, PPL_FP64, at<double>(p, p->a64), p->Nm, p->Pm, p->ldm,
                             at<void>(p, s.am), nullptr));
    }
    return PPL_OK;
  }
  PPL_TRY(convert_rows(p->stream, s.prec, at<double>(p, p->s64), p->Np, p->Pp, p->ldp,
                       at<void>(p, s.sp), s.sp_lo.bytes ? at<void>(p, s.sp_lo) : nullptr));
  if (p->Nm > 0)
    PPL_TRY(convert_rows(p->stream, s.prec, at<double>(p, p->a64), p->Nm, p->Pm, p->ldm,
                         at<void>(p, s.am), s.am_lo.bytes ? at<void>(p, s.am_lo) : nullptr));
  return PPL_OK;
}

// V = (ia|jb) from the occupied-virtual block of L, packed into VS / VA
static int setup_ov_integrals(ppl_plan_t p, const double* L) {
  hipStream_t st = p->stream;
  ProfScope ps(p, PPL_PROF_OTHER, 0.0);
  PPL_TRY(stage_ov(st, L, p->o, p->v, p->naux, p->ldx, at<double>(p, p->xov)));
  const int64_t ov = (int64_t)p->o * p->v;
  double* vfull = at<double>(p, p->g);
  PPL_TRY(gemm_store_f64(st, ov, ov, p->ldx, at<double>(p, p->xov), p->ldx, at<double>(p, p->xov), p->ldx,
                         vfull, ov));
  PPL_TRY(pack_pm(st, p->o, p->v, vfull, (int64_t)p->v * ov, p->v, ov, 1, 0.5, 0.5, 0.5,
                  at<double>(p, p->vs), p->ldp, at<double>(p, p->va), p->ldm, at<int>(p, p->tab_op),
                  at<int>(p, p->tab_om), at<int>(p, p->tab_vp), at<int>(p, p->tab_vm)));
  return PPL_OK;
}

static int read_red(ppl_plan_t p, double out[4]) {
  const double* red_out = at<double>(p, p->red) + kReduceBlocks * 4;
  PPL_HIP_TRY(hipMemcpyAsync(out, red_out, 4 * sizeof(double), hipMemcpyDeviceToHost, p->stream));
  PPL_HIP_TRY(hipStreamSynchronize(p->stream));
  return PPL_OK;
}


// the upper-triangle build relies on symmetric Cholesky vectors (V+- symmetric): PPL_E_ARG
// when the virtual block of L is not symmetric to a relative Frobenius asymmetry of 1e-10
// (synchronous: reads one reduction back)
static int check_symmetric(ppl_plan_t p, const double* L) {
  if (!p->sym_build) return PPL_OK;
  double* partials = at<double>(p, p->red);
  double h[4];
  PPL_TRY(asymmetry_vv(p->stream, L, p->o, p->v, p->naux, partials, partials + kReduceBlocks * 4));
  PPL_TRY(read_red(p, h));
  if (!(h[0] <= 1e-20 * h[1]))
    return fail(PPL_E_ARG, "Cholesky vectors are not symmetric in their virtual block (relative asymmetry %.3g)",
                h[1] > 0.0 ? sqrt(h[0] / h[1]) : 0.0);
  return PPL_OK;
}

// The low-precision V+- of a resident mixed plan, rounded from its complete FP64 copy
// (the same elementwise rounding as the amplitudes before each low-precision sweep): one
// pass over memory instead of a second build in the low precision, and operands closer
// to the FP64 integrals than a low-precision build gives.
static int derive_lowprec(ppl_plan_t p) {
  OperandSet& lo = p->ops[0];
  const OperandSet& f = p->ops[1];
  ProfScope ps(p, PPL_PROF_BUILD_PACK, 0.0);
  PPL_TRY(convert_rows(p->stream, lo.prec, at<double>(p, f.vp), p->Pp, p->Pp, p->ldp, at<void>(p, lo.vp),
                       lo.vp_lo.bytes ? at<void>(p, lo.vp_lo) : nullptr));
  if (p->Pm > 0)
    PPL_TRY(convert_rows(p->stream, lo.prec, at<double>(p, f.vm), p->Pm, p->Pm, p->ldm, at<void>(p, lo.vm),
                         lo.vm_lo.bytes ? at<void>(p, lo.vm_lo) : nullptr));
  lo.built = true;
  return PPL_OK;
}

// ppl_build_batch after its argument and symmetry checks
static int build_checked(ppl_plan_t p, const double* L, int32_t batch) {
  const int nb = (int)p->batches.size();
  p->L_last = L;
  if (!p->resident) return PPL_OK;       // streaming plans build inside ppl_contract
  if (p->ops[1].present) {               // mixed: build in FP64, round to the low precision
    OperandSet& f = p->ops[1];
    if (batch < 0) {
      PPL_TRY(build_all(p, f, L));
      return derive_lowprec(p);
    }
    PPL_TRY(build_one(p, f, L, batch, false));
    if (batch == nb - 1) {
      PPL_TRY(mirror_vpm(p, f));
      f.built = true;
      PPL_TRY(derive_lowprec(p));
    }
    return PPL_OK;
  }
  for (int k = 0; k < 2; ++k) {
    OperandSet& s = p->ops[k];
    if (!s.present) continue;
    if (batch < 0) {
      PPL_TRY(build_all(p, s, L));
    } else {
      PPL_TRY(build_one(p, s, L, batch, false));
      // a resident plan counts as built once its last batch is built in order
      if (batch == nb - 1) {
        PPL_TRY(mirror_vpm(p, s));
        s.built = true;
      }
    }
  }
  return PPL_OK;
}

}  // namespace ppl

using namespace ppl;

static int plan_create(const ppl_desc_t* d, ppl_plan_t* out, bool external_g);

extern "C" {

const char* ppl_last_error(void) { return g_err; }

const char* ppl_version(void) { return "ppl-mi355x 0.1 (gfx950)"; }

int ppl_tile_count(void) { return contract_tile_count(); }

int ppl_tile_dims(int32_t tile, int32_t* bm, int32_t* bn, int32_t* threads) {
  g_err[0] = 0;
  if (!bm || !bn || !threads) return fail(PPL_E_ARG, "NULL output");
  if (tile < 0 || tile >= contract_tile_count()) return fail(PPL_E_ARG, "tile id out of range [0, %d)", contract_tile_count());
  contract_tile_dims(tile, bm, bn, threads);
  return PPL_OK;
}

void ppl_iter_opts_default(ppl_iter_opts_t* o) {
  if (!o) return;
  memset(o, 0, sizeof(*o));
  o->max_sweeps = 100;
  o->start = PPL_START_MP2;
  o->tol = 1e-7;
  o->switch_tol = 0.0;
  o->stagnation = 0.95;
  o->min_fp64_sweeps = 2;
  o->fail_on_noconv = 1;
  o->diverge_factor = 1e3;
  o->history = nullptr;
  o->diis = 0;
  o->hhl = 0;
  o->ring = 0;
}

int ppl_plan(const ppl_desc_t* d, ppl_plan_t* out) { return plan_create(d, out, false); }

}  // extern "C"

// ppl_plan; with external_g the plan's layout leaves out its build scratch, which the caller
// places and assigns (p->g) before the workspace is bound
static int plan_create(const ppl_desc_t* d, ppl_plan_t* out, bool external_g) {
  g_err[0] = 0;
  if (!d || !out) return fail(PPL_E_ARG, "null argument");
  *out = nullptr;
  if (d->o < 1) return fail(PPL_E_ARG, "o must be >= 1 (got %d)", d->o);
  if (d->v < 2) return fail(PPL_E_ARG, "v must be >= 2 (got %d)", d->v);
  if (d->naux < 1) return fail(PPL_E_ARG, "naux must be >= 1 (got %d)", d->naux);
  if (d->v > 32767 || d->o > 32767) return fail(PPL_E_ARG, "o and v must be < 32768");
  if (d->prec != PPL_FP64 && d->prec != PPL_FP32 && d->prec != PPL_BF16X3 && d->prec != PPL_BF16X6)
    return fail(PPL_E_ARG, "unknown precision %d", d->prec);
  if (d->tile_contract < -1 || d->tile_contract >= contract_tile_count())
    return fail(PPL_E_ARG, "tile_contract %d out of range", d->tile_contract);
  if (d->diis_max < 0 || d->diis_max > PPL_DIIS_MAX)
    return fail(PPL_E_ARG, "diis_max %d out of range [0, %d]", d->diis_max, PPL_DIIS_MAX);
  if (d->flags & ~(PPL_PLAN_CONTRACT_ONLY | PPL_PLAN_RING)) return fail(PPL_E_ARG, "unknown plan flags 0x%x", d->flags);
  if ((d->flags & PPL_PLAN_CONTRACT_ONLY) && (d->flags & PPL_PLAN_RING))
    return fail(PPL_E_ARG, "PPL_PLAN_RING serves the iteration, which a PPL_PLAN_CONTRACT_ONLY plan cannot run");
  // 64-bit size sanity: the largest products used anywhere
  {
    uint64_t x;
    const uint64_t v = d->v, o = d->o, na = d->naux;
    const uint64_t Pp = v * (v + 1) / 2;
    if (!mul_ok(Pp, Pp, &x) || !mul_ok(x, 16, &x) || !mul_ok(v * v, na + 64, &x) ||
        !mul_ok(x, 16, &x) || !mul_ok(o * o, v * v, &x) || !mul_ok(x, 16, &x))
      return fail(PPL_E_ARG, "sizes overflow 64-bit byte counts");
  }
  ppl_plan_t p = new (std::nothrow) ppl_plan_s();
  if (!p) return fail(PPL_E_NOMEM, "host allocation failed");
  p->g_external = external_g;
  p->o = d->o;
  p->v = d->v;
  p->naux = d->naux;
  p->prec = d->prec;
  p->keep_fp64 = (d->prec != PPL_FP64) && d->keep_fp64;
  p->contract_only = (d->flags & PPL_PLAN_CONTRACT_ONLY) != 0;
  p->ring = (d->flags & PPL_PLAN_RING) != 0;
  p->diis_max = p->contract_only ? 0 : d->diis_max;
  p->stream = (hipStream_t)d->stream;
  p->Pp = npairs_plus(p->v);
  p->Pm = npairs_minus(p->v);
  p->Np = npairs_plus(p->o);
  p->Nm = npairs_minus(p->o);
  p->ldp = pad_ld(p->Pp);
  p->ldm = pad_ld(std::max<int64_t>(p->Pm, 1));
  p->ldx = pad_ld(p->naux);
  p->ops[0].prec = p->prec;
  p->ops[0].present = true;
  p->ops[1].prec = PPL_FP64;
  p->ops[1].present = p->keep_fp64 != 0;
  p->tile_build = build_tile_for_prec(p->prec);
  p->tile_build64 = p->ops[1].present ? build_tile_for_prec(PPL_FP64) : p->tile_build;
  {
    int t = d->tile_contract, sp = 1;
    contract_choose(p->prec, p->Np, p->Pp, p->ldp, kMaxSplits, &t, &sp);
    p->tile_contract = t;
    p->split_p = sp;
    t = -1;
    sp = 1;
    if (p->Nm > 0) contract_choose(p->prec, p->Nm, p->Pm, p->ldm, kMaxSplits, &t, &sp);
    p->tile_m = t < 0 ? 0 : t;
    p->split_m = sp;
    if (p->ops[1].present) {   // the FP64 copy gets the model's choice for FP64 operands
      OperandSet& f = p->ops[1];
      t = -1;
      sp = 1;
      contract_choose(PPL_FP64, p->Np, p->Pp, p->ldp, kMaxSplits, &t, &sp);
      f.tile_p = t;
      f.split_p = sp;
      t = -1;
      sp = 1;
      if (p->Nm > 0) contract_choose(PPL_FP64, p->Nm, p->Pm, p->ldm, kMaxSplits, &t, &sp);
      f.tile_m = t < 0 ? 0 : t;
      f.split_m = sp;
    }
  }

  if (d->tune_cache) p->tune_cache = d->tune_cache;
  if (d->tile_contract < 0) {
    int cfg[4];
    if (tune_cache_lookup(p->tune_cache, p->prec, p->o, p->v, p->ldp, p->ldm, cfg)) {
      p->tile_contract = cfg[0];
      p->split_p = cfg[1];
      p->tile_m = cfg[2];
      p->split_m = cfg[3];
    }
  }

  uint64_t budget = d->hbm_budget;
  if (budget == 0) {
    size_t fr = 0, tot = 0;
    hipError_t e = hipMemGetInfo(&fr, &tot);
    if (e != hipSuccess) {
      delete p;
      return fail(PPL_E_HIP, "hipMemGetInfo failed: %s (pass an explicit hbm_budget)", hipGetErrorString(e));
    }
    budget = (uint64_t)(0.9 * (double)fr);
  }
  p->budget = budget;

  // G cap: at most build_scratch (default 4 GiB) of scratch, at least one full row a = 0 (v pairs)
  const uint64_t per_pair_g = (uint64_t)p->v * p->v * g_acc_bytes(p);
  const uint64_t gbytes_cap = d->build_scratch ? d->build_scratch : (4ull << 30);
  int64_t gcap = (int64_t)std::max<uint64_t>((uint64_t)p->v, gbytes_cap / per_pair_g);
  gcap = std::min<int64_t>(gcap, p->Pp);
  // try resident (V+- symmetric: build the upper triangle, mirror the rest; PPL_SYM_BUILD=0
  // builds every row in full instead)
  {
    const char* e = getenv("PPL_SYM_BUILD");
    p->sym_build = !(e && e[0] == '0');
  }
  make_batches(p->v, gcap, p->batches);
  make_tile_tables(p);
  uint64_t need = assign_layout(p, gcap, true, 0);
  if (need <= budget) {
    p->resident = true;
    if (p->sym_build) build_column_order(p->v, p->cols_host);
  } else {
    // streaming: upper-triangle steps contracted as U and U^T (FP64 plans with one operand set)
    p->sym_build = p->sym_build && p->prec == PPL_FP64 && !p->keep_fp64;
    // streaming: V+- rows of one build step at a time; the largest step that fits
    // (the need grows with the step's pair count, so a bisection over it suffices)
    p->resident = false;
    auto need_for = [&](int64_t cap) {
      make_batches(p->v, cap, p->batches);
      make_tile_tables(p);
      int64_t maxp = 0;
      for (const Batch& b : p->batches) maxp = std::max<int64_t>(maxp, b.p1 - b.p0);
      return assign_layout(p, cap, false, maxp);
    };
    int64_t lo = std::min<int64_t>(p->v, gcap), hi = gcap;
    need = need_for(lo);
    if (need > budget) {
      const uint64_t n2 = need;
      delete p;
      return fail(PPL_E_NOMEM, "budget %llu B cannot hold one V+- row batch (needs %llu B)",
                  (unsigned long long)budget, (unsigned long long)n2);
    }
    if (hi > lo && need_for(hi) <= budget) {
      lo = hi;
    } else {
      while (hi - lo > std::max<int64_t>(1, lo / 32)) {
        const int64_t mid = lo + (hi - lo) / 2;
        if (need_for(mid) <= budget) lo = mid;
        else hi = mid;
      }
    }
    need = need_for(lo);
    gcap = lo;
    if (p->sym_build) build_column_order(p->v, p->cols_host);
  }
  p->g_pairs_cap = gcap;
  p->a_per_batch = p->batches.empty() ? 0 : p->batches[0].a1 - p->batches[0].a0;
  p->ws_bytes_needed = need;
  *out = p;
  return PPL_OK;
}

extern "C" {

int ppl_plan_query(ppl_plan_t p, ppl_plan_info_t* info) {
  PPL_TRY(check_plan(p));
  if (!info) return fail(PPL_E_ARG, "null info");
  memset(info, 0, sizeof(*info));
  info->workspace_bytes = p->ws_bytes_needed;
  uint64_t vpm = 0;
  for (int k = 0; k < 2; ++k)
    if (p->ops[k].present)
      vpm += ((uint64_t)p->Pp * p->ldp + (uint64_t)p->Pm * p->ldm) * elem_bytes(p->ops[k].prec) *
             planes(p->ops[k].prec);
  info->vpm_bytes = vpm;
  info->n_batches = (int32_t)p->batches.size();
  info->resident = p->resident ? 1 : 0;
  info->a_per_batch = p->a_per_batch;
  info->tile_build = p->tile_build;
  info->tile_contract = p->tile_contract;
  info->n_plus = (int32_t)p->Np;
  info->n_minus = (int32_t)p->Nm;
  info->p_plus = (int32_t)p->Pp;
  info->p_minus = (int32_t)p->Pm;
  info->splits_contract = p->split_p;
  info->build_scratch_bytes = p->g.bytes;
  {
    int64_t mp = 0;
    for (const Batch& b : p->batches) mp = std::max<int64_t>(mp, b.p1 - b.p0);
    info->max_step_pairs = mp;
  }
  info->tile_contract_minus = p->tile_m;
  info->splits_contract_minus = p->split_m;
  info->flops_build = build_flops(p, 0, p->v);
  info->flops_contract =
      2.0 * ((double)p->Pp * p->Pp * p->Np + (double)p->Pm * p->Pm * p->Nm);
  return PPL_OK;
}

int ppl_bind_workspace(ppl_plan_t p, void* dptr, uint64_t bytes) {
  g_err[0] = 0;
  PPL_TRY(check_plan(p));
  if (!dptr) return fail(PPL_E_ARG, "null workspace");
  if (((uintptr_t)dptr) % 256 != 0) return fail(PPL_E_ARG, "workspace must be 256-byte aligned");
  if (bytes < p->ws_bytes_needed)
    return fail(PPL_E_NOMEM, "workspace of %llu B is smaller than the %llu B the plan needs",
                (unsigned long long)bytes, (unsigned long long)p->ws_bytes_needed);
  PPL_HIP_TRY(hipGetDevice(&p->device));
  p->ws = (char*)dptr;
  p->ws_bytes = bytes;
  for (int k = 0; k < 2; ++k) p->ops[k].built = false;
  hipStream_t st = p->stream;
  // zero every small region (amplitude rows, results, integrals (ia|jb)): their padding must stay 0
  const Region* small[] = {&p->ops[0].sp, &p->ops[0].am, &p->ops[0].sp_lo, &p->ops[0].am_lo,
                           &p->ops[1].sp, &p->ops[1].am, &p->rp,          &p->rm,
                           &p->s64,       &p->a64,       &p->vs,          &p->va};
  for (const Region* r : small)
    if (r->bytes) PPL_TRY(zero_bytes(st, p->ws + r->off, r->bytes));
  PPL_TRY(fill_tables(st, p->o, p->v, at<int>(p, p->tab_vp), at<int>(p, p->tab_vm), at<int>(p, p->tab_op),
                      at<int>(p, p->tab_om)));
  if (!p->tiles_host.empty())
    PPL_HIP_TRY(hipMemcpyAsync(at<int>(p, p->tiles), p->tiles_host.data(), p->tiles_host.size() * 4,
                               hipMemcpyHostToDevice, st));
  if (p->sym_build)
    PPL_HIP_TRY(hipMemcpyAsync(at<int>(p, p->cols), p->cols_host.data(), p->cols_host.size() * 4,
                               hipMemcpyHostToDevice, st));
  std::vector<int64_t> cube_off;
  if (p->cube_off.bytes) {
    cube_off.assign((size_t)p->v + 1, 0);
    for (int a = 0; a < p->v; ++a) cube_off[a + 1] = cube_off[a] + cubes_of(p->v, a);
    PPL_HIP_TRY(hipMemcpyAsync(at<int64_t>(p, p->cube_off), cube_off.data(), cube_off.size() * 8,
                               hipMemcpyHostToDevice, st));
  }
  PPL_HIP_TRY(hipStreamSynchronize(st));   // the host tile table must not be reused before the copy ends
  p->setup_done = true;
  return PPL_OK;
}

int ppl_build_batch(ppl_plan_t p, const double* L, int32_t batch) {
  g_err[0] = 0;
  PPL_TRY(check_bound(p));
  if (!L) return fail(PPL_E_ARG, "null L");
  const int nb = (int)p->batches.size();
  if (batch < -1 || batch >= nb) return fail(PPL_E_ARG, "batch %d out of range [-1, %d)", batch, nb);
  if (batch <= 0) PPL_TRY(check_symmetric(p, L));
  return build_checked(p, L, batch);
}

}  // extern "C"


namespace ppl {
// (ki|lj) from the occupied block of L and W+-_{ij,kl} = ((ki|lj) +- (li|kj)) / 2 on the
// i<=j (i<j) rows and k<=l (k<l) columns, in the hole-hole scratch
static int hhl_integrals(ppl_plan_t p, const double* L) {
  const HhlScratch h = hhl_scratch(p);
  char* g = at<char>(p, p->g);
  double *xoo = (double*)(g + h.xoo), *woo = (double*)(g + h.woo);
  const int64_t o = p->o, oo = o * o;
  const int *tab_op = at<int>(p, p->tab_op), *tab_om = at<int>(p, p->tab_om);
  PPL_TRY(stage_oo(p->stream, L, p->o, p->v, p->naux, p->ldx, xoo));
  PPL_TRY(gemm_store_f64(p->stream, oo, oo, p->ldx, xoo, p->ldx, xoo, p->ldx, woo, oo));
  // X_ij^kl = Woo[(k,i)][(l,j)]
  return pack_pm(p->stream, p->o, p->o, woo, oo, 1, o * oo, o, 0.5, 0.5, 0.5, (double*)(g + h.wp), h.ldq,
                 (double*)(g + h.wm), h.ldqm, tab_op, tab_om, tab_op, tab_om);
}

// The hole-hole ladder of packed amplitudes X (S' rows [N+][ldp] or A' rows [N-][ldm],
// FP64), one chunk of virtual pairs at a time: the chunk's columns of X transposed into
// sT (S' scaled by (2 - d_kl)/(2 - d_ab)), C = sT W^T with K = the occupied pairs, then
// C^T added into the same columns of the results (add: R rows of the operand set's
// accumulator type) or written over the chunk's columns of X itself (!add).
static int hhl_pass(ppl_plan_t p, const HhlScratch& h, bool plus, double* X, void* R, int rprec, bool add) {
  char* g = at<char>(p, p->g);
  hipStream_t st = p->stream;
  const int64_t Nq = plus ? p->Np : p->Nm, Pq = plus ? p->Pp : p->Pm;
  const int64_t ldx = plus ? p->ldp : p->ldm, ldk = plus ? h.ldq : h.ldqm;
  if (Nq <= 0 || Pq <= 0) return PPL_OK;
  const int* tab_q = at<int>(p, p->tab_op);
  const int* tab_p = at<int>(p, p->tab_vp);
  double* sT = (double*)(g + h.st);
  double* C = (double*)(g + h.cp);
  const double* W = (const double*)(g + (plus ? h.wp : h.wm));
  for (int64_t p0 = 0; p0 < Pq; p0 += h.chunk) {
    const int64_t np = std::min<int64_t>(h.chunk, Pq - p0);
    PPL_TRY(transpose_pm(st, X + p0, ldx, sT, ldk, Nq, np, plus ? tab_q : nullptr, plus ? tab_p + p0 : nullptr,
                         plus ? 1 : 0));
    int tile = -1, sp = 1;
    contract_choose(PPL_FP64, np, Nq, ldk, 1, &tile, &sp);
    PPL_TRY(gemm_contract(st, PPL_FP64, tile, np, Nq, ldk, sT, nullptr, ldk, W, nullptr, ldk, C, ldk, 0, 1, nullptr,
                          ldk, 0));
    if (add)
      PPL_TRY(add_transposed(st, rprec, (char*)R + p0 * (rprec == PPL_FP64 ? 8 : 4), ldx, C, ldk, Nq, np));
    else
      PPL_TRY(transpose_pm(st, C, ldk, X + p0, ldx, np, Nq, nullptr, nullptr, 0, 0));
  }
  return PPL_OK;
}

// R+- += the hole-hole ladder of the packed amplitudes S'/A' (FP64 masters), in the
// accumulator type of the operand set's results
static int hhl_add_packed(ppl_plan_t p, const OperandSet& s) {
  const HhlScratch h = hhl_scratch(p, p->g.bytes);
  const int cprec = s.prec == PPL_FP64 ? PPL_FP64 : PPL_FP32;
  PPL_TRY(hhl_pass(p, h, true, at<double>(p, p->s64), at<void>(p, p->rp), cprec, true));
  return hhl_pass(p, h, false, at<double>(p, p->a64), at<void>(p, p->rm), cprec, true);
}

static int contract_impl(ppl_plan_t p, const double* t2, const double* t1, double* R, double alpha,
                         double beta) {
  g_err[0] = 0;
  PPL_TRY(check_bound(p));
  if (!t2 || !R) return fail(PPL_E_ARG, "null t2 or R");
  if ((const void*)t2 == (const void*)R) return fail(PPL_E_ARG, "R may not alias t2");
  OperandSet& s = p->ops[0];
  const int64_t o = p->o, v = p->v;
  // S' = (2 - d_cd)(t^cd + t^dc)/2, A' = t^cd - t^dc on the i<=j / i<j rows (t + t1 t1 with singles)
  PPL_TRY(pack_pm(p->stream, p->o, p->v, t2, o * v * v, v * v, v, 1, 1.0, 0.5, 1.0, at<double>(p, p->s64),
                  p->ldp, at<double>(p, p->a64), p->ldm, at<int>(p, p->tab_op), at<int>(p, p->tab_om),
                  at<int>(p, p->tab_vp), at<int>(p, p->tab_vm), t1));
  PPL_TRY(refresh_operands(p, s));
  PPL_TRY(contract_packed(p, s));
  PPL_TRY(unpack_r(p->stream, s.prec == PPL_FP64 ? PPL_FP64 : PPL_FP32, p->o, p->v, at<void>(p, p->rp),
                   p->ldp, at<void>(p, p->rm), p->ldm, R, alpha, beta));
  return PPL_OK;
}
}  // namespace ppl

extern "C" {

int ppl_contract(ppl_plan_t p, const double* t2, double* R, double alpha, double beta) {
  return contract_impl(p, t2, nullptr, R, alpha, beta);
}

int ppl_contract_tau(ppl_plan_t p, const double* t2, const double* t1, double* R, double alpha, double beta) {
  if (!t1) return fail(PPL_E_ARG, "null t1");
  return contract_impl(p, t2, t1, R, alpha, beta);
}

int ppl_hhl(ppl_plan_t p, const double* L, const double* t2, double* R, double alpha, double beta) {
  g_err[0] = 0;
  PPL_TRY(check_bound(p));
  if (!L || !t2 || !R) return fail(PPL_E_ARG, "null device pointer");
  if ((const void*)t2 == (const void*)R) return fail(PPL_E_ARG, "R may not alias t2");
  const HhlScratch h = hhl_scratch(p);
  if (h.bytes > p->g.bytes)
    return fail(PPL_E_STATE, "hole-hole scratch needs %llu B, the plan has %llu B",
                (unsigned long long)h.bytes, (unsigned long long)p->g.bytes);
  const int64_t o = p->o, v = p->v;
  ProfScope ps(p, PPL_PROF_OTHER, 2.0 * (double)p->Pp * p->Np * p->Np + 2.0 * (double)p->Pm * p->Nm * p->Nm);
  hipStream_t st = p->stream;
  double* s64 = at<double>(p, p->s64);
  double* a64 = at<double>(p, p->a64);
  PPL_TRY(hhl_integrals(p, L));
  // S'/A' of t2 into the FP64 packed rows, the ladder chunk by chunk over the virtual
  // pairs written back over them, then unpacked
  PPL_TRY(pack_pm(st, p->o, p->v, t2, o * v * v, v * v, v, 1, 1.0, 0.5, 1.0, s64, p->ldp, a64, p->ldm,
                  at<int>(p, p->tab_op), at<int>(p, p->tab_om), at<int>(p, p->tab_vp), at<int>(p, p->tab_vm)));
  const HhlScratch hs = hhl_scratch(p, p->g.bytes);
  PPL_TRY(hhl_pass(p, hs, true, s64, nullptr, PPL_FP64, false));
  PPL_TRY(hhl_pass(p, hs, false, a64, nullptr, PPL_FP64, false));
  return unpack_r(st, PPL_FP64, p->o, p->v, s64, p->ldp, a64, p->ldm, R, alpha, beta);
}

// J[(k,c)][(j,b)] = (kc|jb) and K[(k,c)][(j,b)] = (kj|bc) from L (scratch w laid out by r)
static int ring_integrals(hipStream_t st, int o, int v, int naux, const double* L, char* w, const RingLayout& r) {
  auto d = [&](uint64_t off) { return (double*)(w + off); };
  const int64_t ov = (int64_t)o * v;
  // the K-dimension padding of J and K must read as zero (their GEMMs write n < o v only)
  PPL_TRY(zero_bytes(st, w + r.j, 2 * (uint64_t)ov * r.ldk * 8));
  PPL_TRY(stage_ov(st, L, o, v, naux, r.ldx, d(r.xov)));
  PPL_TRY(stage_oo(st, L, o, v, naux, r.ldx, d(r.xoo)));
  PPL_TRY(stage_vv(st, PPL_FP64, L, o, v, naux, r.ldx, d(r.xvv), nullptr));
  // J[(k,c)][(j,b)] = sum_P L^P_kc L^P_jb;  G[(k,j)][(b,c)] = sum_P L^P_kj L^P_bc -> K
  PPL_TRY(gemm_store_f64(st, ov, ov, r.ldx, d(r.xov), r.ldx, d(r.xov), r.ldx, d(r.j), r.ldk));
  PPL_TRY(gemm_store_f64(st, (int64_t)o * o, (int64_t)v * v, r.ldx, d(r.xoo), r.ldx, d(r.xvv), r.ldx, d(r.g),
                         r.ldg));
  return ring_exchange(st, o, v, d(r.g), r.ldg, d(r.k), r.ldk);
}

// R = beta R + alpha RING(t2) with J and K already in the scratch
static int ring_apply(hipStream_t st, int o, int v, const double* t2, double* R, double alpha, double beta, char* w,
                      const RingLayout& r) {
  auto d = [&](uint64_t off) { return (double*)(w + off); };
  const int64_t ov = (int64_t)o * v;
  PPL_TRY(ring_pack(st, o, v, t2, r.ldk, d(r.xa), d(r.an), d(r.b)));
  // C1 = Xa J^T + An K^T, C2 = B K^T (J and K are symmetric: their rows are their columns)
  int tile = -1, sp = 1;
  contract_choose(PPL_FP64, ov, ov, r.ldk, 1, &tile, &sp);
  PPL_TRY(gemm_contract(st, PPL_FP64, tile, ov, ov, r.ldk, d(r.xa), nullptr, r.ldk, d(r.j), nullptr, r.ldk,
                        d(r.c1), r.ldk, 0, 1, nullptr, 0, 0, false));
  PPL_TRY(gemm_contract(st, PPL_FP64, tile, ov, ov, r.ldk, d(r.an), nullptr, r.ldk, d(r.k), nullptr, r.ldk,
                        d(r.c1), r.ldk, 0, 1, nullptr, 0, 0, true));
  PPL_TRY(gemm_contract(st, PPL_FP64, tile, ov, ov, r.ldk, d(r.b), nullptr, r.ldk, d(r.k), nullptr, r.ldk,
                        d(r.c2), r.ldk, 0, 1, nullptr, 0, 0, false));
  return ring_unpack(st, o, v, d(r.c1), d(r.c2), r.ldk, R, alpha, beta);
}

// J and K of the scratch (FP64, from ring_integrals) in the low precision of the layout
static int ring_integrals_lp(hipStream_t st, int o, int v, char* w, const RingLayout& r) {
  const int64_t ov = (int64_t)o * v;
  const int prec = r.lp_prec;
  PPL_TRY(convert_rows(st, prec, (const double*)(w + r.j), ov, ov, r.ldk, w + r.jl,
                       prec == PPL_FP32 ? nullptr : w + r.jl + r.lp_plane));
  return convert_rows(st, prec, (const double*)(w + r.k), ov, ov, r.ldk, w + r.kl,
                      prec == PPL_FP32 ? nullptr : w + r.kl + r.lp_plane);
}

// R = RING(t2) with the three GEMMs in the layout's low precision (FP32 accumulation): the
// operands are packed in that precision into the Xa, An and B regions (FP64-sized, so they
// hold every plane), the FP32 results C1, C2 go to their FP64-sized regions.
static int ring_apply_lp(hipStream_t st, int o, int v, const double* t2, double* R, char* w, const RingLayout& r) {
  const int64_t ov = (int64_t)o * v;
  const int prec = r.lp_prec;
  const uint64_t pl = r.lp_plane;
  auto lo = [&](uint64_t off) -> void* { return prec == PPL_FP32 ? nullptr : (void*)(w + off + pl); };
  PPL_TRY(ring_pack_lp(st, prec, o, v, t2, r.ldk, w + r.xa, lo(r.xa), w + r.an, lo(r.an), w + r.b, lo(r.b)));
  int tile = -1, sp = 1;
  contract_choose(prec, ov, ov, r.ldk, 1, &tile, &sp);
  float* c1 = (float*)(w + r.c1);
  float* c2 = (float*)(w + r.c2);
  PPL_TRY(gemm_contract(st, prec, tile, ov, ov, r.ldk, w + r.xa, lo(r.xa), r.ldk, w + r.jl, lo(r.jl), r.ldk, c1,
                        r.ldk, 0, 1, nullptr, 0, 0, false));
  PPL_TRY(gemm_contract(st, prec, tile, ov, ov, r.ldk, w + r.an, lo(r.an), r.ldk, w + r.kl, lo(r.kl), r.ldk, c1,
                        r.ldk, 0, 1, nullptr, 0, 0, true));
  PPL_TRY(gemm_contract(st, prec, tile, ov, ov, r.ldk, w + r.b, lo(r.b), r.ldk, w + r.kl, lo(r.kl), r.ldk, c2,
                        r.ldk, 0, 1, nullptr, 0, 0, false));
  return ring_unpack_f32(st, o, v, c1, c2, r.ldk, R, 1.0, 0.0);
}

uint64_t ppl_ring_scratch_bytes(int32_t o, int32_t v, int32_t naux) {
  RingLayout r;
  return ring_layout(o, v, naux, r) ? r.bytes : 0;
}

int ppl_ring(int32_t o, int32_t v, int32_t naux, const double* L, const double* t2, double* R, double alpha,
             double beta, void* scratch, uint64_t scratch_bytes, void* stream) {
  g_err[0] = 0;
  RingLayout r;
  if (!ring_layout(o, v, naux, r)) return fail(PPL_E_ARG, "bad sizes o=%d v=%d naux=%d", o, v, naux);
  if (!L || !t2 || !R || !scratch) return fail(PPL_E_ARG, "null device pointer");
  if ((const void*)t2 == (const void*)R) return fail(PPL_E_ARG, "R may not alias t2");
  if ((uintptr_t)scratch % 256 != 0) return fail(PPL_E_ARG, "scratch must be 256-byte aligned");
  if (scratch_bytes < r.bytes)
    return fail(PPL_E_ARG, "ring scratch holds %llu B, needs %llu B", (unsigned long long)scratch_bytes,
                (unsigned long long)r.bytes);
  hipStream_t st = (hipStream_t)stream;
  PPL_TRY(ring_integrals(st, o, v, naux, L, (char*)scratch, r));
  return ring_apply(st, o, v, t2, R, alpha, beta, (char*)scratch, r);
}

}  // extern "C"

// ---------------------------------------------------------------- ring terms without allocation
// Scratch of ppl_ring_static: one file-scope device array, a copy of which every GPU the
// library runs on holds until the process ends. Host code never uses its name as an
// address: the device address of each GPU's copy comes from hipGetSymbolAddress, taken
// once per device (with that device current) on the first call there and kept below.
static __device__ __align__(256) char g_static_scratch[PPL_RING_STATIC_BYTES];

constexpr int kMaxDevices = 64;
static std::mutex g_static_mu;
static void* g_static_ptr[kMaxDevices] = {};

// device address of the current device's copy of g_static_scratch; the stream (if any)
// must belong to the current device
static int static_scratch(hipStream_t st, void** out) {
  int dev = 0;
  PPL_HIP_TRY(hipGetDevice(&dev));
  if (st) {
    int sdev = -1;
    PPL_HIP_TRY(hipStreamGetDevice(st, &sdev));
    if (sdev != dev)
      return fail(PPL_E_ARG, "the stream belongs to device %d, the current device is %d", sdev, dev);
  }
  if (dev < 0 || dev >= kMaxDevices) return fail(PPL_E_UNSUPPORTED, "device id %d out of range", dev);
  std::lock_guard<std::mutex> lock(g_static_mu);
  if (!g_static_ptr[dev]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(g_static_scratch));
    if (e != hipSuccess || !ptr)
      return fail(PPL_E_HIP, "hipGetSymbolAddress of the static scratch failed on device %d: %s", dev,
                  hipGetErrorString(e));
    g_static_ptr[dev] = ptr;
  }
  *out = g_static_ptr[dev];
  return PPL_OK;
}

extern "C" {

int ppl_ring_static(int32_t o, int32_t v, int32_t naux, const double* L, const double* t2, double* R,
                    double alpha, double beta, void* stream) {
  g_err[0] = 0;
  RingLayout r;
  if (!ring_layout(o, v, naux, r)) return fail(PPL_E_ARG, "bad sizes o=%d v=%d naux=%d", o, v, naux);
  if (!L || !t2 || !R) return fail(PPL_E_ARG, "null device pointer");
  if ((const void*)t2 == (const void*)R) return fail(PPL_E_ARG, "R may not alias t2");
  if (r.bytes > (uint64_t)PPL_RING_STATIC_BYTES)
    return fail(PPL_E_ARG,
                "the ring terms at o=%d v=%d naux=%d need %llu B of scratch, more than the %llu B static "
                "scratch (use ppl_ring with a caller scratch)",
                o, v, naux, (unsigned long long)r.bytes, (unsigned long long)PPL_RING_STATIC_BYTES);
  hipStream_t st = (hipStream_t)stream;
  void* ws = nullptr;
  PPL_TRY(static_scratch(st, &ws));
  // the same kernels as ppl_ring, on this device's copy of the static scratch
  PPL_TRY(ring_integrals(st, o, v, naux, L, (char*)ws, r));
  return ring_apply(st, o, v, t2, R, alpha, beta, (char*)ws, r);
}

int ppl_iterate(ppl_plan_t p, const double* L, const double* e_occ, const double* e_vir, double* t2,
                const ppl_iter_opts_t* opts, ppl_iter_report_t* rep) {
  g_err[0] = 0;
  PPL_TRY(check_bound(p));
  if (p->contract_only) return fail(PPL_E_STATE, "a PPL_PLAN_CONTRACT_ONLY plan cannot iterate");
  if (!L || !e_occ || !e_vir || !t2) return fail(PPL_E_ARG, "null device pointer");
  ppl_iter_opts_t o;
  if (opts) o = *opts; else ppl_iter_opts_default(&o);
  if (o.max_sweeps < 1) return fail(PPL_E_ARG, "max_sweeps must be >= 1");
  if (o.start < PPL_START_MP2 || o.start > PPL_START_GIVEN_CHECKED) return fail(PPL_E_ARG, "bad start");
  if (o.hhl && !p->resident)
    return fail(PPL_E_UNSUPPORTED, "the hole-hole ladder in the iteration needs a resident plan");
  if (o.hhl && hhl_scratch(p).bytes > p->g.bytes) return fail(PPL_E_STATE, "hole-hole scratch too small");
  if (o.ring && (!p->ring || !p->resident))
    return fail(PPL_E_STATE, "the ring terms in the iteration need a resident plan made with PPL_PLAN_RING");
  if (o.diis < 0 || o.diis > p->diis_max)
    return fail(PPL_E_ARG, "diis %d exceeds the plan's subspace capacity %d (ppl_desc_t.diis_max)", o.diis,
                p->diis_max);
  ppl_iter_report_t r;
  memset(&r, 0, sizeof(r));
  hipStream_t st = p->stream;
  double* partials = at<double>(p, p->red);
  double* red_out = partials + kReduceBlocks * 4;
  double h[4];

  // integrals: V = (ia|jb) packed into VS / VA, then V+- of every operand set, then the
  // hole-hole W+- (the build scratch holds them for the sweeps of a resident plan)
  PPL_TRY(setup_ov_integrals(p, L));
  PPL_TRY(ppl_build_batch(p, L, -1));
  if (o.hhl) PPL_TRY(hhl_integrals(p, L));
  RingLayout rl;
  if (o.ring) {
    ring_layout(p->o, p->v, p->naux, rl, p->ops[0].prec);
    PPL_TRY(ring_integrals(st, p->o, p->v, p->naux, L, at<char>(p, p->ring_ws), rl));
    if (rl.lp_prec != PPL_FP64) PPL_TRY(ring_integrals_lp(st, p->o, p->v, at<char>(p, p->ring_ws), rl));
  }

  const int* tabs[4] = {at<int>(p, p->tab_op), at<int>(p, p->tab_om), at<int>(p, p->tab_vp),
                        at<int>(p, p->tab_vm)};
  double* s64 = at<double>(p, p->s64);
  double* a64 = at<double>(p, p->a64);
  auto load_mp2 = [&]() -> int {
    return mp2_start(st, p->o, p->v, e_occ, e_vir, at<double>(p, p->vs), at<double>(p, p->va), p->ldp,
                     p->ldm, s64, a64, tabs[0], tabs[1], tabs[2], tabs[3], partials, red_out);
  };
  auto load_given = [&]() -> int {
    return pack_pm(st, p->o, p->v, t2, (int64_t)p->o * p->v * p->v, (int64_t)p->v * p->v, p->v, 1, 1.0,
                   0.5, 1.0, s64, p->ldp, a64, p->ldm, tabs[0], tabs[1], tabs[2], tabs[3]);
  };
  if (o.start == PPL_START_MP2) PPL_TRY(load_mp2());
  else PPL_TRY(load_given());
  PPL_TRY(energy_only(st, p->o, p->v, at<double>(p, p->vs), at<double>(p, p->va), s64, a64, p->ldp, p->ldm,
                      tabs[0], tabs[1], tabs[2], tabs[3], partials, red_out));
  PPL_TRY(read_red(p, h));
  r.energy_start = h[1];
  if ((h[2] != 0.0 || !isfinite(h[1])) && o.start == PPL_START_GIVEN_CHECKED) {
    // a checked guess with NaN or Inf entries is rejected before any sweep: the
    // iteration falls back to the MP2 start, which the checked start promises
    PPL_TRY(load_mp2());
    PPL_TRY(energy_only(st, p->o, p->v, at<double>(p, p->vs), at<double>(p, p->va), s64, a64, p->ldp, p->ldm,
                        tabs[0], tabs[1], tabs[2], tabs[3], partials, red_out));
    PPL_TRY(read_red(p, h));
    r.energy_start = h[1];
    r.restarted_mp2 = 1;
    o.start = PPL_START_MP2;
  }
  if (h[2] != 0.0 || !isfinite(h[1])) {
    r.status = PPL_E_NONFINITE;
    if (rep) *rep = r;
    return fail(PPL_E_NONFINITE, "non-finite start amplitudes");
  }

  // which operand set a sweep uses
  const bool mixed = p->ops[0].prec != PPL_FP64;
  // automatic switch point: a few times above the rounding floor of the low-precision GEMMs
  // (relative single-evaluation errors ~3e-6 for BF16x3 and ~2e-7 for FP32)
  if (o.switch_tol <= 0.0) o.switch_tol = p->ops[0].prec == PPL_BF16X3 ? 1e-6 : 1e-7;
  const int fp64_set = mixed ? (p->ops[1].present ? 1 : -1) : 0;
  bool lp_phase = mixed;
  int fp64_sweeps = 0;
  double r_prev = -1.0, r_first = -1.0;
  int status = PPL_E_NOCONV;
  int sweeps = 0;

  // DIIS state: slot ids of the subspace (oldest first), their inner products, and the
  // slot the current sweep writes (-1: a plain sweep)
  const bool diis_on = o.diis >= 2;
  std::vector<int> sub;
  double B[kDiisMax][kDiisMax] = {};
  int slot = -1;
  double* const dT = diis_on ? at<double>(p, p->diis_t) : nullptr;
  double* const dE = diis_on ? at<double>(p, p->diis_e) : nullptr;
  double* const dred = diis_on ? at<double>(p, p->diis_red) : nullptr;

  auto sweep_once = [&](OperandSet& s) -> int {
    PPL_TRY(refresh_operands(p, s));
    PPL_TRY(contract_packed(p, s));
    if (o.hhl) {
      ProfScope ph(p, PPL_PROF_OTHER, 2.0 * (double)p->Pp * p->Np * p->Np + 2.0 * (double)p->Pm * p->Nm * p->Nm);
      PPL_TRY(hhl_add_packed(p, s));
    }
    if (o.ring) {
      // the ring terms of the current FP64 amplitudes, added to R+- in their precision
      const double ov = (double)p->o * p->v;
      ProfScope pr(p, PPL_PROF_OTHER, 6.0 * ov * ov * ov);
      PPL_TRY(unpack_t(st, p->o, p->v, s64, p->ldp, a64, p->ldm, at<double>(p, p->tfull)));
      if (s.prec == PPL_FP64)
        PPL_TRY(ring_apply(st, p->o, p->v, at<double>(p, p->tfull), at<double>(p, p->rfull), 1.0, 0.0,
                           at<char>(p, p->ring_ws), rl));
      else   // low-precision sweeps: the ring GEMMs in the sweep's precision as well
        PPL_TRY(ring_apply_lp(st, p->o, p->v, at<double>(p, p->tfull), at<double>(p, p->rfull),
                              at<char>(p, p->ring_ws), rl));
      PPL_TRY(add_pm(st, s.prec == PPL_FP64 ? PPL_FP64 : PPL_FP32, p->o, p->v, at<double>(p, p->rfull),
                     at<void>(p, p->rp), p->ldp, at<void>(p, p->rm), p->ldm, tabs[0], tabs[1], tabs[2], tabs[3]));
    }
    ProfScope ps(p, PPL_PROF_UPDATE, 0.0);
    double* ts = slot >= 0 ? dT + slot * p->diis_slot_n : nullptr;
    double* es = slot >= 0 ? dE + slot * p->diis_slot_n : nullptr;
    PPL_TRY(update_sweep(st, s.prec == PPL_FP64 ? PPL_FP64 : PPL_FP32, p->o, p->v, e_occ, e_vir,
                         at<double>(p, p->vs), at<double>(p, p->va), at<void>(p, p->rp), at<void>(p, p->rm),
                         p->ldp, p->ldm, s64, a64, tabs[0], tabs[1], tabs[2], tabs[3], partials, red_out,
                         ts, es));
    return read_red(p, h);
  };
  // before a DIIS sweep: the slot it writes (the oldest vector's once the subspace is full)
  auto diis_pick_slot = [&]() {
    if ((int)sub.size() == o.diis) sub.erase(sub.begin());
    for (int k = 0; k < o.diis; ++k)
      if (std::find(sub.begin(), sub.end(), k) == sub.end()) {
        slot = k;
        return;
      }
  };
  // after it: add the new vector, extrapolate the next input into S'/A'
  auto diis_step = [&]() -> int {
    ProfScope ps(p, PPL_PROF_UPDATE, 0.0);
    sub.push_back(slot);
    DiisSet set{};
    set.n = (int)sub.size();
    for (int i = 0; i < set.n; ++i) set.id[i] = sub[i];
    PPL_TRY(diis_dots(st, p->o, p->v, p->ldp, p->ldm, tabs[0], tabs[1], tabs[2], tabs[3], dE, p->diis_slot_n,
                      set, slot, dred, dred + kReduceBlocks * kDiisMax));
    double dots[kDiisMax];
    PPL_HIP_TRY(hipMemcpyAsync(dots, dred + kReduceBlocks * kDiisMax, set.n * sizeof(double),
                               hipMemcpyDeviceToHost, st));
    PPL_HIP_TRY(hipStreamSynchronize(st));
    for (int i = 0; i < set.n; ++i) B[slot][sub[i]] = B[sub[i]][slot] = dots[i];
    double c[kDiisMax];
    while (!diis_solve(B, sub, c)) {
      if (sub.size() == 1) {   // a zero error vector: the sweep's own amplitudes
        c[0] = 1.0;
        break;
      }
      sub.erase(sub.begin());
      ++r.diis_dropped;
    }
    set.n = (int)sub.size();
    for (int i = 0; i < set.n; ++i) {
      set.id[i] = sub[i];
      set.c[i] = c[i];
    }
    slot = -1;
    return diis_combine(st, p->o, p->v, p->ldp, p->ldm, dT, p->diis_slot_n, set, s64, a64);
  };
  auto count_sweep = [&](const OperandSet& s, double rr) {
    if (o.history && sweeps < o.max_sweeps) o.history[sweeps] = rr;
    ++sweeps;
    if (s.prec == PPL_FP64) { ++r.sweeps_fp64; ++fp64_sweeps; } else { ++r.sweeps_lp; }
    r.residual = rr;
    r.energy = h[1];
  };

  // A checked start runs the first sweep from the given amplitudes and from MP2
  // and keeps whichever has the smaller first residual (both sweeps count).
  if (o.start == PPL_START_GIVEN_CHECKED && o.max_sweeps >= 2) {
    OperandSet& s0 = (lp_phase || fp64_set < 0) ? p->ops[0] : p->ops[fp64_set];
    PPL_TRY(sweep_once(s0));
    const double r_given = sqrt(fabs(h[0]));
    const double e_given = h[1];
    const bool given_ok = h[2] == 0.0 && isfinite(r_given);
    count_sweep(s0, r_given);
    // keep the given start's first iterate
    PPL_TRY(convert_rows(st, PPL_FP64, s64, p->Np, p->Pp, p->ldp, at<void>(p, p->bs), nullptr));
    if (p->Nm > 0) PPL_TRY(convert_rows(st, PPL_FP64, a64, p->Nm, p->Pm, p->ldm, at<void>(p, p->ba), nullptr));
    PPL_TRY(load_mp2());
    PPL_TRY(sweep_once(s0));
    const double r_mp2 = sqrt(fabs(h[0]));
    count_sweep(s0, r_mp2);
    if (given_ok && r_given <= r_mp2) {
      PPL_TRY(convert_rows(st, PPL_FP64, at<double>(p, p->bs), p->Np, p->Pp, p->ldp, s64, nullptr));
      if (p->Nm > 0) PPL_TRY(convert_rows(st, PPL_FP64, at<double>(p, p->ba), p->Nm, p->Pm, p->ldm, a64, nullptr));
      r.residual = r_given;
      r.energy = e_given;
    } else {
      r.restarted_mp2 = 1;
    }
    r_first = r.residual;
    r_prev = r.residual;
  }

  while (sweeps < o.max_sweeps) {
    OperandSet& s = (lp_phase || fp64_set < 0) ? p->ops[0] : p->ops[fp64_set];
    if (diis_on) diis_pick_slot();
    PPL_TRY(sweep_once(s));
    const double rr = sqrt(fabs(h[0]));
    count_sweep(s, rr);
    if (r_first < 0) r_first = rr;
    if (h[2] != 0.0 || !isfinite(rr) || !isfinite(h[1])) { status = PPL_E_NONFINITE; break; }
    if (o.diverge_factor > 0 && rr > o.diverge_factor * r_first) { status = PPL_E_DIVERGED; break; }
    bool restart = false;
    if (lp_phase) {
      const bool stagnant = r_prev > 0 && rr / r_prev > o.stagnation;
      if (fp64_set >= 0 && (rr < o.switch_tol || stagnant)) {
        lp_phase = false;
        restart = true;
      }
      else if (fp64_set < 0 && o.tol > 0 && rr < o.tol) { status = PPL_OK; break; }
    } else {
      const int need = mixed ? o.min_fp64_sweeps : 0;
      if (o.tol > 0 && rr < o.tol && fp64_sweeps >= need) { status = PPL_OK; break; }
    }
    r_prev = rr;
    if (diis_on && sweeps < o.max_sweeps) {
      if (restart) {     // FP64 sweeps start a new subspace from this sweep's amplitudes
        sub.clear();
        slot = -1;
      } else {
        PPL_TRY(diis_step());
      }
    }
  }
  if (o.tol <= 0 && status == PPL_E_NOCONV) status = PPL_OK;   // fixed sweep count requested
  PPL_TRY(unpack_t(st, p->o, p->v, s64, p->ldp, a64, p->ldm, t2));
  PPL_HIP_TRY(hipStreamSynchronize(st));
  r.status = status;
  if (rep) *rep = r;
  if (status == PPL_E_NOCONV && !o.fail_on_noconv) return PPL_OK;
  if (status != PPL_OK)
    return fail(status, "iteration ended with status %d after %d sweeps (residual %.3e)", status, sweeps,
                r.residual);
  return PPL_OK;
}

int ppl_set_contract_config(ppl_plan_t p, int32_t tp, int32_t sp, int32_t tm, int32_t sm) {
  PPL_TRY(check_plan(p));
  const int nt = contract_tile_count();
  if (tp < 0 || tp >= nt || tm < 0 || tm >= nt) return fail(PPL_E_ARG, "tile id out of range [0, %d)", nt);
  if (sp < 0 || sp > kMaxSplits || sm < 0 || sm > kMaxSplits)
    return fail(PPL_E_ARG, "split count out of range [0, %d] (0 = stream-K)", kMaxSplits);
  p->tile_contract = tp;
  p->split_p = sp;
  p->tile_m = tm;
  p->split_m = sm;
  return PPL_OK;
}

int ppl_autotune(ppl_plan_t p, int32_t reps, double* best_ms) { return autotune_impl(p, reps, best_ms); }

}  // extern "C"

namespace ppl {
int autotune_impl(ppl_plan_t p, int32_t reps, double* best_ms) {
  g_err[0] = 0;
  PPL_TRY(check_bound(p));
  if (reps < 1) return fail(PPL_E_ARG, "reps must be >= 1");
  OperandSet& s = p->ops[0];
  if (!p->resident || !s.built) return fail(PPL_E_STATE, "autotune needs a resident plan with V+- built");
  hipStream_t st = p->stream;
  hipEvent_t e0, e1;
  PPL_HIP_TRY(hipEventCreate(&e0));
  PPL_HIP_TRY(hipEventCreate(&e1));
  void* part = at<void>(p, p->part);
  const int nt = contract_tile_count();
  double best[2] = {1e300, 1e300};
  int bt[2] = {p->tile_contract, p->tile_m}, bs[2] = {p->split_p, p->split_m};
  int rc = PPL_OK;
  for (int which = 0; which < 2 && rc == PPL_OK; ++which) {
    const bool plus = which == 0;
    const int64_t Nr = plus ? p->Np : p->Nm, Pr = plus ? p->Pp : p->Pm, ld = plus ? p->ldp : p->ldm;
    if (Nr <= 0 || Pr <= 0) continue;
    const void* A = at<void>(p, plus ? s.sp : s.am);
    const void* A_lo = (plus ? s.sp_lo : s.am_lo).bytes ? at<void>(p, plus ? s.sp_lo : s.am_lo) : nullptr;
    const void* V = at<void>(p, plus ? s.vp : s.vm);
    const void* V_lo = (plus ? s.vp_lo : s.vm_lo).bytes ? at<void>(p, plus ? s.vp_lo : s.vm_lo) : nullptr;
    void* C = at<void>(p, plus ? p->rp : p->rm);
    auto run = [&](int t, int sp) {
      return gemm_contract(st, s.prec, t, Nr, Pr, ld, A, A_lo, ld, V, V_lo, ld, C, ld, 0, sp, part, ld, p->part.bytes);
    };
    // average over n launches after one untimed launch
    auto timed = [&](int t, int sp, int n, double& ms_out) {
      PPL_TRY(run(t, sp));
      PPL_HIP_TRY(hipEventRecord(e0, st));
      for (int r = 0; r < n; ++r) PPL_TRY(run(t, sp));
      float ms = 0.f;
      PPL_HIP_TRY(hipEventRecord(e1, st));
      PPL_HIP_TRY(hipEventSynchronize(e1));
      PPL_HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
      ms_out = ms / n;
      return PPL_OK;
    };
    // bring the device to its steady clock before the first candidate is timed
    for (int r = 0; r < 8 && rc == PPL_OK; ++r) rc = run(plus ? p->tile_contract : p->tile_m, 1);
    // every (tile, K decomposition): split counts 1 .. kMaxSplits, then stream-K (0)
    struct Cand { double ms; int t, sp; };
    std::vector<Cand> cands;
    for (int t = 0; t < nt && rc == PPL_OK; ++t)
      for (int k = 1; k <= kMaxSplits + 1 && rc == PPL_OK; ++k) {
        const int sp = k <= kMaxSplits ? k : 0;
        // BF16x6 keeps its K slices short (accuracy); stream-K ranges are not bounded
        if (s.prec == PPL_BF16X6 && (sp == 0 || sp < contract_min_splits(s.prec, ld))) continue;
        if (sp > 1 && contract_jobs(t, s.prec, Nr, Pr, ld, sp) == contract_jobs(t, s.prec, Nr, Pr, ld, sp - 1))
          continue;   // same effective split count as a smaller request
        double ms = 0.0;
        rc = timed(t, sp, reps, ms);
        cands.push_back({ms, t, sp});
      }
    if (rc != PPL_OK) break;
    // the four fastest again, interleaved over three rounds, so that a slow or fast
    // moment of the device does not decide alone
    std::sort(cands.begin(), cands.end(), [](const Cand& x, const Cand& y) { return x.ms < y.ms; });
    const size_t nf = std::min<size_t>(4, cands.size());
    std::vector<double> tot(nf, 0.0);
    for (int round = 0; round < 3 && rc == PPL_OK; ++round)
      for (size_t c = 0; c < nf && rc == PPL_OK; ++c) {
        double ms = 0.0;
        rc = timed(cands[c].t, cands[c].sp, reps, ms);
        tot[c] += ms;
      }
    if (rc != PPL_OK) break;
    for (size_t c = 0; c < nf; ++c)
      if (tot[c] / 3.0 < best[which]) {
        best[which] = tot[c] / 3.0;
        bt[which] = cands[c].t;
        bs[which] = cands[c].sp;
      }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (rc != PPL_OK) return rc;
  p->tile_contract = bt[0];
  p->split_p = bs[0];
  p->tile_m = bt[1];
  p->split_m = bs[1];
  if (!p->tune_cache.empty()) {
    const int cfg[4] = {bt[0], bs[0], bt[1], bs[1]};
    PPL_TRY(tune_cache_append(p->tune_cache, p->prec, p->o, p->v, cfg));
  }
  if (best_ms) {
    best_ms[0] = best[0] < 1e300 ? best[0] : 0.0;
    best_ms[1] = best[1] < 1e300 ? best[1] : 0.0;
  }
  return PPL_OK;
}
}  // namespace ppl

extern "C" {

int ppl_profile_enable(ppl_plan_t p, int on) {
  PPL_TRY(check_plan(p));
  if (on) {
    if (p->prof_next > 0) PPL_HIP_TRY(hipStreamSynchronize(p->stream));
    p->prof_recs.clear();
    p->prof_next = 0;
  }
  p->prof_on = on != 0;
  return PPL_OK;
}

int ppl_profile_read(ppl_plan_t p, ppl_profile_t* out) {
  PPL_TRY(check_plan(p));
  if (!out) return fail(PPL_E_ARG, "null profile");
  memset(out, 0, sizeof(*out));
  PPL_HIP_TRY(hipStreamSynchronize(p->stream));
  for (const auto& r : p->prof_recs) {
    float ms = 0.f;
    PPL_HIP_TRY(hipEventElapsedTime(&ms, p->prof_pool[r.ev], p->prof_pool[r.ev + 1]));
    out->launches[r.kind] += 1;
    out->ms[r.kind] += ms;
    out->flops[r.kind] += r.flops;
  }
  return PPL_OK;
}

int ppl_mp2(ppl_plan_t p, const double* L, const double* e_occ, const double* e_vir, double* t2_out,
            double* e_mp2) {
  g_err[0] = 0;
  PPL_TRY(check_bound(p));
  if (p->contract_only) return fail(PPL_E_STATE, "a PPL_PLAN_CONTRACT_ONLY plan has no (ia|jb) buffers");
  if (!L || !e_occ || !e_vir || !t2_out) return fail(PPL_E_ARG, "null device pointer");
  hipStream_t st = p->stream;
  double* partials = at<double>(p, p->red);
  double* red_out = partials + kReduceBlocks * 4;
  PPL_TRY(setup_ov_integrals(p, L));
  double* s64 = at<double>(p, p->s64);
  double* a64 = at<double>(p, p->a64);
  PPL_TRY(mp2_start(st, p->o, p->v, e_occ, e_vir, at<double>(p, p->vs), at<double>(p, p->va), p->ldp, p->ldm,
                    s64, a64, at<int>(p, p->tab_op), at<int>(p, p->tab_om), at<int>(p, p->tab_vp),
                    at<int>(p, p->tab_vm), partials, red_out));
  PPL_TRY(unpack_t(st, p->o, p->v, s64, p->ldp, a64, p->ldm, t2_out));
  if (e_mp2) {
    double h[4];
    PPL_TRY(read_red(p, h));
    *e_mp2 = h[1];
  }
  return PPL_OK;
}

int ppl_mlp_sigma(ppl_plan_t p, const double* t_mp2, double* sigma) {
  g_err[0] = 0;
  PPL_TRY(check_bound(p));
  if (!t_mp2 || !sigma) return fail(PPL_E_ARG, "null pointer");
  double* partials = at<double>(p, p->red);
  double* red_out = partials + kReduceBlocks * 4;
  const int64_t n = (int64_t)p->o * p->o * p->v * p->v;
  PPL_TRY(sumsq_launch(p->stream, t_mp2, n, partials, red_out));
  double h[4];
  PPL_TRY(read_red(p, h));
  *sigma = sqrt(h[0] / (double)n);
  return PPL_OK;
}

int ppl_mlp_samples(ppl_plan_t p, const double* t_mp2, const double* t_star, const double* e_occ,
                    const double* e_vir, double sigma, const int64_t* idx, int64_t n, float* X, float* Y) {
  g_err[0] = 0;
  PPL_TRY(check_bound(p));
  if (!t_mp2 || !e_occ || !e_vir || !idx || !X || n < 0) return fail(PPL_E_ARG, "bad argument");
  if ((t_star == nullptr) != (Y == nullptr)) return fail(PPL_E_ARG, "t_star and Y go together");
  if (!(sigma > 0.0)) return fail(PPL_E_ARG, "sigma must be > 0");
  if (n == 0) return PPL_OK;
  return mlp_samples_launch(p->stream, p->o, p->v, t_mp2, t_star, e_occ, e_vir, sigma, idx, n, X, Y);
}

int ppl_destroy(ppl_plan_t p) {
  if (!p) return PPL_OK;
  for (hipEvent_t e : p->prof_pool) (void)hipEventDestroy(e);
  delete p;
  return PPL_OK;
}

// ---------------------------------------------------------------- learned start
}  // extern "C"

struct ppl_mlp_s {
  hipStream_t stream = nullptr;
  int64_t max_batch = 0;
  char* ws = nullptr;
  uint64_t ws_bytes = 0, need = 0;
  ppl::Region prm, m, v, grad, gpart, lpart, loss;
  int step = 0;
};

namespace ppl {
template <class T>
inline T* mat(ppl_mlp_t q, const Region& r) {
  return reinterpret_cast<T*>(q->ws + r.off);
}
static int mlp_check(ppl_mlp_t q) {
  if (!q) return fail(PPL_E_ARG, "null mlp");
  if (!q->ws) return fail(PPL_E_STATE, "no MLP workspace bound");
  return PPL_OK;
}
// splitmix64: a small published counter-based generator for the host-side init
static uint64_t splitmix64(uint64_t& x) {
  uint64_t z = (x += 0x9E3779B97F4A7C15ull);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}
}  // namespace ppl

extern "C" {

int ppl_mlp_create(int32_t width, int64_t max_batch, void* stream, ppl_mlp_t* out) {
  g_err[0] = 0;
  if (!out) return fail(PPL_E_ARG, "null out");
  *out = nullptr;
  if (width != 128) return fail(PPL_E_UNSUPPORTED, "only width 128 is built (got %d)", width);
  if (max_batch < 1 || max_batch > (int64_t)1 << 26) return fail(PPL_E_ARG, "max_batch out of range");
  ppl_mlp_t q = new (std::nothrow) ppl_mlp_s();
  if (!q) return fail(PPL_E_NOMEM, "host allocation failed");
  q->stream = (hipStream_t)stream;
  q->max_batch = max_batch;
  const uint64_t P = (uint64_t)mlp_param_count();
  const uint64_t nwg = (uint64_t)((max_batch + mlp_train_rows() - 1) / mlp_train_rows());
  Layout L;
  q->prm = L.take(P * 4);
  q->m = L.take(P * 4);
  q->v = L.take(P * 4);
  q->grad = L.take(P * 4);
  q->gpart = L.take(nwg * P * 4);
  q->lpart = L.take(nwg * 4);
  q->loss = L.take(16);
  q->need = L.cur;
  *out = q;
  return PPL_OK;
}

int ppl_mlp_workspace_bytes(ppl_mlp_t q, uint64_t* bytes) {
  if (!q || !bytes) return fail(PPL_E_ARG, "null argument");
  *bytes = q->need;
  return PPL_OK;
}

int ppl_mlp_param_count(ppl_mlp_t q) {
  (void)q;
  return mlp_param_count();
}

int ppl_mlp_bind_workspace(ppl_mlp_t q, void* dptr, uint64_t bytes) {
  g_err[0] = 0;
  if (!q || !dptr) return fail(PPL_E_ARG, "null argument");
  if (((uintptr_t)dptr) % 256 != 0) return fail(PPL_E_ARG, "workspace must be 256-byte aligned");
  if (bytes < q->need) return fail(PPL_E_NOMEM, "MLP workspace needs %llu bytes", (unsigned long long)q->need);
  q->ws = (char*)dptr;
  q->ws_bytes = bytes;
  PPL_TRY(zero_bytes(q->stream, q->ws, q->need));
  q->step = 0;
  return PPL_OK;
}

int ppl_mlp_set_params(ppl_mlp_t q, const float* host, int64_t n) {
  g_err[0] = 0;
  PPL_TRY(mlp_check(q));
  if (!host || n != mlp_param_count()) return fail(PPL_E_ARG, "expected %d parameters", mlp_param_count());
  PPL_HIP_TRY(hipMemcpyAsync(mat<float>(q, q->prm), host, (size_t)n * 4, hipMemcpyHostToDevice, q->stream));
  PPL_TRY(zero_bytes(q->stream, q->ws + q->m.off, q->m.bytes));
  PPL_TRY(zero_bytes(q->stream, q->ws + q->v.off, q->v.bytes));
  PPL_HIP_TRY(hipStreamSynchronize(q->stream));
  q->step = 0;
  return PPL_OK;
}

int ppl_mlp_get_params(ppl_mlp_t q, float* host, int64_t n) {
  g_err[0] = 0;
  PPL_TRY(mlp_check(q));
  if (!host || n != mlp_param_count()) return fail(PPL_E_ARG, "expected %d parameters", mlp_param_count());
  PPL_HIP_TRY(hipMemcpyAsync(host, mat<float>(q, q->prm), (size_t)n * 4, hipMemcpyDeviceToHost, q->stream));
  PPL_HIP_TRY(hipStreamSynchronize(q->stream));
  return PPL_OK;
}

int ppl_mlp_init(ppl_mlp_t q, uint64_t seed) {
  g_err[0] = 0;
  PPL_TRY(mlp_check(q));
  const int P = mlp_param_count(), H = 128;
  std::vector<float> w(P);
  uint64_t st = seed;
  auto uni = [&](double bound) {
    const double u = (double)(splitmix64(st) >> 11) * (1.0 / 9007199254740992.0);   // [0, 1)
    return (float)((2.0 * u - 1.0) * bound);
  };
  int o = 0;
  for (int k = 0; k < H * 4; ++k) w[o++] = uni(1.0 / sqrt(4.0));     // W1
  for (int k = 0; k < H; ++k) w[o++] = uni(1.0 / sqrt(4.0));         // b1
  for (int k = 0; k < H * H; ++k) w[o++] = uni(1.0 / sqrt((double)H));  // W2
  for (int k = 0; k < H; ++k) w[o++] = uni(1.0 / sqrt((double)H));     // b2
  for (int k = 0; k < H; ++k) w[o++] = uni(1.0 / sqrt((double)H));     // W3
  w[o++] = uni(1.0 / sqrt((double)H));                                  // b3
  return ppl_mlp_set_params(q, w.data(), P);
}

int ppl_mlp_grad(ppl_mlp_t q, const float* X, const float* Y, int64_t n, float* host_grad, float* host_loss) {
  g_err[0] = 0;
  PPL_TRY(mlp_check(q));
  if (!X || !Y || n < 1 || n > q->max_batch) return fail(PPL_E_ARG, "bad batch (n = %lld)", (long long)n);
  PPL_TRY(mlp_train_launch(q->stream, mat<float>(q, q->prm), X, Y, n, mat<float>(q, q->gpart),
                           mat<float>(q, q->lpart), mat<float>(q, q->grad), mat<float>(q, q->loss)));
  if (host_grad)
    PPL_HIP_TRY(hipMemcpyAsync(host_grad, mat<float>(q, q->grad), (size_t)mlp_param_count() * 4,
                               hipMemcpyDeviceToHost, q->stream));
  if (host_loss)
    PPL_HIP_TRY(hipMemcpyAsync(host_loss, mat<float>(q, q->loss), 4, hipMemcpyDeviceToHost, q->stream));
  PPL_HIP_TRY(hipStreamSynchronize(q->stream));
  return PPL_OK;
}

int ppl_mlp_train_step(ppl_mlp_t q, const float* X, const float* Y, int64_t n, float lr, float* host_loss) {
  g_err[0] = 0;
  PPL_TRY(mlp_check(q));
  if (!X || !Y || n < 1 || n > q->max_batch) return fail(PPL_E_ARG, "bad batch (n = %lld)", (long long)n);
  if (!(lr > 0.0f)) return fail(PPL_E_ARG, "lr must be > 0");
  PPL_TRY(mlp_train_launch(q->stream, mat<float>(q, q->prm), X, Y, n, mat<float>(q, q->gpart),
                           mat<float>(q, q->lpart), mat<float>(q, q->grad), mat<float>(q, q->loss)));
  q->step += 1;
  PPL_TRY(mlp_adam_launch(q->stream, mat<float>(q, q->prm), mat<float>(q, q->grad), mat<float>(q, q->m),
                          mat<float>(q, q->v), lr, q->step, 0.9f, 0.999f, 1e-8f));
  if (host_loss) {
    PPL_HIP_TRY(hipMemcpyAsync(host_loss, mat<float>(q, q->loss), 4, hipMemcpyDeviceToHost, q->stream));
    PPL_HIP_TRY(hipStreamSynchronize(q->stream));
  }
  return PPL_OK;
}

int ppl_mlp_guess(ppl_mlp_t q, ppl_plan_t p, const double* t_mp2, const double* e_occ, const double* e_vir,
                  double sigma, double* t2_out) {
  g_err[0] = 0;
  PPL_TRY(mlp_check(q));
  PPL_TRY(check_bound(p));
  if (!t_mp2 || !e_occ || !e_vir || !t2_out) return fail(PPL_E_ARG, "null device pointer");
  if ((const void*)t_mp2 == (const void*)t2_out) return fail(PPL_E_ARG, "t2_out may not alias t_mp2");
  if (!(sigma > 0.0)) return fail(PPL_E_ARG, "sigma must be > 0");
  return mlp_infer_launch(p->stream, mat<float>(q, q->prm), p->o, p->v, t_mp2, e_occ, e_vir, sigma,
                          at<int>(p, p->tab_om), at<int>(p, p->tab_vp), t2_out);
}

int ppl_mlp_destroy(ppl_mlp_t q) {
  delete q;
  return PPL_OK;
}

// ---------------------------------------------------------------- batched instances
}  // extern "C"

struct ppl_batch_s {
  int n = 0, prec = PPL_FP64;
  hipStream_t stream = nullptr;
  std::vector<ppl_plan_t> plans;
  std::vector<uint64_t> offs;
  uint64_t need = 0;
  ppl::Region groups_r, items_r, counter_r;   // counter_r: queue counters, then the queue starts
  std::vector<int> q_begin;                   // host copy of the queue starts (kept for the async copy)
  int64_t max_items = 0;
  char* ws = nullptr;
  std::vector<ppl::GroupDesc> groups;
  std::vector<int4> items;
  std::vector<int> gtile;                     // grouped tile per instance GEMM (2k: R+, 2k+1: R-), -1 = model
  bool built = false, prepared = false;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  // integral builds of the instances run as concurrent branches, one per side stream, each a
  // longest-first share of the instances; fork and join through events on the batch stream
  static constexpr int kBranches = 4;
  int n_branches = kBranches;                 // PPL_BATCH_BRANCHES (1 .. kBranches) at plan time
  hipStream_t side[kBranches] = {};
  hipEvent_t ev_fork = nullptr, ev_join[kBranches] = {};
  std::vector<int> branch_of;                 // instance -> branch
  ppl::Region g_branch[kBranches];            // the build scratch each branch's instances share
};

namespace ppl {
static int batch_check(ppl_batch_t b) {
  if (!b) return fail(PPL_E_ARG, "null batch");
  if (!b->ws) return fail(PPL_E_STATE, "no batch workspace bound");
  return PPL_OK;
}


// byte offset of the queue start table inside the batch's counter region
constexpr uint64_t kQueueBeginOffset = 64;
static_assert(kGroupedQueues * sizeof(int) <= kQueueBeginOffset &&
              kQueueBeginOffset + (kGroupedQueues + 1) * sizeof(int) <= 256, "counter region layout");

static int batch_prepare(ppl_batch_t b) {
  b->groups.clear();
  b->items.clear();
  const int KC = kc_of_prec(b->prec);
  // a column group: every row tile of one column tile of one instance GEMM (they read
  // the same V rows, so they go to one XCD queue and are handed out back to back)
  struct Col { int gi; int n0, bm; int64_t M; double work; };
  std::vector<Col> cols;
  int64_t n_items = 0;
  for (int k = 0; k < b->n; ++k) {
    ppl_plan_t p = b->plans[k];
    OperandSet& s = p->ops[0];
    for (int which = 0; which < 2; ++which) {
      const bool plus = which == 0;
      const int64_t M = plus ? p->Np : p->Nm, N = plus ? p->Pp : p->Pm, ld = plus ? p->ldp : p->ldm;
      if (M <= 0 || N <= 0) continue;
      const int forced = (int)b->gtile.size() > 2 * k + which ? b->gtile[2 * k + which] : -1;
      const int tile = forced >= 0 ? forced : grouped_choose_tile(b->prec, M);
      GroupDesc g;
      g.a_off = at<char>(p, plus ? s.sp : s.am) - b->ws;
      g.b_off = at<char>(p, plus ? s.vp : s.vm) - b->ws;
      g.c_off = at<char>(p, plus ? p->rp : p->rm) - b->ws;
      g.M = M;
      g.N = N;
      g.nk = ld / KC;
      g.lda = g.ldb = g.ldc = ld;
      g.cfg = tile;
      g.pad = 0;
      const int gi = (int)b->groups.size();
      b->groups.push_back(g);
      int bm, bn;
      grouped_tile_dims(tile, &bm, &bn);
      const int64_t n_mt = (M + bm - 1) / bm;
      for (int64_t nt = 0; nt * bn < N; ++nt) {
        cols.push_back({gi, (int)(nt * bn), bm, M, (double)n_mt * bm * bn * g.nk});
        n_items += n_mt;
      }
    }
  }
  if (n_items > b->max_items) return fail(PPL_E_ARG, "too many batch items");
  // longest column groups first, each to the least loaded queue; a queue runs its
  // groups in that order
  std::stable_sort(cols.begin(), cols.end(), [](const Col& x, const Col& y) { return x.work > y.work; });
  std::vector<std::vector<int4>> q(kGroupedQueues);
  double load[kGroupedQueues] = {0};
  for (const Col& c : cols) {
    int qi = 0;
    for (int j = 1; j < kGroupedQueues; ++j)
      if (load[j] < load[qi]) qi = j;
    for (int64_t m0 = 0; m0 < c.M; m0 += c.bm) q[qi].push_back(int4{c.gi, (int)m0, c.n0, 0});
    load[qi] += c.work;
  }
  b->q_begin.assign(1, 0);
  for (int j = 0; j < kGroupedQueues; ++j) {
    b->items.insert(b->items.end(), q[j].begin(), q[j].end());
    b->q_begin.push_back((int)b->items.size());
  }
  if (!b->groups.empty())
    PPL_HIP_TRY(hipMemcpyAsync(b->ws + b->groups_r.off, b->groups.data(), b->groups.size() * sizeof(GroupDesc),
                               hipMemcpyHostToDevice, b->stream));
  if (!b->items.empty())
    PPL_HIP_TRY(hipMemcpyAsync(b->ws + b->items_r.off, b->items.data(), b->items.size() * sizeof(int4),
                               hipMemcpyHostToDevice, b->stream));
  PPL_HIP_TRY(hipMemcpyAsync(b->ws + b->counter_r.off + kQueueBeginOffset, b->q_begin.data(),
                             b->q_begin.size() * sizeof(int), hipMemcpyHostToDevice, b->stream));
  PPL_HIP_TRY(hipStreamSynchronize(b->stream));
  b->prepared = true;
  return PPL_OK;
}

static int batch_enqueue(ppl_batch_t b, const double* const* t2, double* const* R) {
  for (int k = 0; k < b->n; ++k) {
    ppl_plan_t p = b->plans[k];
    const int64_t o = p->o, v = p->v;
    if (!t2[k] || !R[k]) return fail(PPL_E_ARG, "null t2 or R for instance %d", k);
    PPL_TRY(pack_pm(b->stream, p->o, p->v, t2[k], o * v * v, v * v, v, 1, 1.0, 0.5, 1.0, at<double>(p, p->s64),
                    p->ldp, at<double>(p, p->a64), p->ldm, at<int>(p, p->tab_op), at<int>(p, p->tab_om),
                    at<int>(p, p->tab_vp), at<int>(p, p->tab_vm)));
    PPL_TRY(refresh_operands(p, p->ops[0]));
  }
  const int n_items = (int)b->items.size();
  const int grid = n_items < 512 ? n_items : 512;
  PPL_TRY(gemm_grouped(b->stream, b->prec, b->ws, reinterpret_cast<const GroupDesc*>(b->ws + b->groups_r.off),
                       reinterpret_cast<const int4*>(b->ws + b->items_r.off), n_items,
                       reinterpret_cast<const int*>(b->ws + b->counter_r.off + kQueueBeginOffset),
                       reinterpret_cast<int*>(b->ws + b->counter_r.off), grid));
  for (int k = 0; k < b->n; ++k) {
    ppl_plan_t p = b->plans[k];
    PPL_TRY(unpack_r(b->stream, b->prec == PPL_FP64 ? PPL_FP64 : PPL_FP32, p->o, p->v, at<void>(p, p->rp),
                     p->ldp, at<void>(p, p->rm), p->ldm, R[k], 1.0, 0.0));
  }
  return PPL_OK;
}

// Integral builds of every instance (staging, build steps, mirror) from L[k]; no host
// synchronization (the symmetry of each L was checked by the eager ppl_batch_build). With
// branches the builds are forked from the batch stream over the side streams and joined
// back into it; without, they run in turn on the batch stream. Graph capture takes the
// latter: replays of a captured graph with such branches left their workspace unreleased
// after the graph and its memory were freed (measured: about one workspace per replayed
// graph), which a single-stream graph does not.
static int batch_build_branches(ppl_batch_t b, const double* const* L, bool branches) {
  if (b->n_branches == 1 || !branches) {    // every build on the batch stream
    for (int k = 0; k < b->n; ++k) PPL_TRY(build_checked(b->plans[k], L[k], -1));
    return PPL_OK;
  }
  if (!b->ev_fork) {
    PPL_HIP_TRY(hipEventCreateWithFlags(&b->ev_fork, hipEventDisableTiming));
    for (int j = 0; j < ppl_batch_s::kBranches; ++j) {
      PPL_HIP_TRY(hipStreamCreateWithFlags(&b->side[j], hipStreamNonBlocking));
      PPL_HIP_TRY(hipEventCreateWithFlags(&b->ev_join[j], hipEventDisableTiming));
    }
  }
  PPL_HIP_TRY(hipEventRecord(b->ev_fork, b->stream));
  for (int j = 0; j < ppl_batch_s::kBranches; ++j) PPL_HIP_TRY(hipStreamWaitEvent(b->side[j], b->ev_fork, 0));
  int rc = PPL_OK;
  for (int k = 0; k < b->n && rc == PPL_OK; ++k) {
    ppl_plan_t p = b->plans[k];
    hipStream_t own = p->stream;
    p->stream = b->side[b->branch_of[k]];
    rc = build_checked(p, L[k], -1);
    p->stream = own;
  }
  // join every branch, also after a failure, so that the stream leaves no fork open
  for (int j = 0; j < ppl_batch_s::kBranches; ++j) {
    PPL_HIP_TRY(hipEventRecord(b->ev_join[j], b->side[j]));
    PPL_HIP_TRY(hipStreamWaitEvent(b->stream, b->ev_join[j], 0));
  }
  return rc;
}

static void batch_drop_graph(ppl_batch_t b) {
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  b->exec = nullptr;
  b->graph = nullptr;
}
}  // namespace ppl

extern "C" {

int ppl_batch_plan(int32_t n, const ppl_desc_t* descs, ppl_batch_t* out) {
  g_err[0] = 0;
  if (!out || !descs || n < 1) return fail(PPL_E_ARG, "bad batch arguments");
  *out = nullptr;
  const int prec = descs[0].prec;
  if (prec != PPL_FP64 && prec != PPL_FP32) return fail(PPL_E_UNSUPPORTED, "batched instances run in FP64 or FP32");
  ppl_batch_t b = new (std::nothrow) ppl_batch_s();
  if (!b) return fail(PPL_E_NOMEM, "host allocation failed");
  b->n = n;
  b->prec = prec;
  b->stream = (hipStream_t)descs[0].stream;
  uint64_t off = 0;
  int64_t max_items = 0;
  for (int k = 0; k < n; ++k) {
    ppl_desc_t d = descs[k];
    if (d.prec != prec || d.stream != descs[0].stream) {
      ppl_batch_destroy(b);
      return fail(PPL_E_ARG, "all instances need the same precision and stream");
    }
    d.keep_fp64 = 0;
    d.diis_max = 0;                      // batched instances are contracted, not iterated
    d.flags |= PPL_PLAN_CONTRACT_ONLY;
    if (d.hbm_budget == 0) d.hbm_budget = (uint64_t)1 << 62;
    // the instances of one build branch build in turn and share one scratch (placed below)
    if (d.build_scratch == 0) d.build_scratch = (uint64_t)2 << 30;
    ppl_plan_t p = nullptr;
    const int rc = plan_create(&d, &p, true);
    if (rc != PPL_OK) {
      ppl_batch_destroy(b);
      return rc;
    }
    b->plans.push_back(p);
    if (!p->resident) {
      ppl_batch_destroy(b);
      return fail(PPL_E_UNSUPPORTED, "instance %d does not fit its budget resident", k);
    }
    b->offs.push_back(off);
    off += align256(p->ws_bytes_needed);
    // upper bound of items: the smallest grouped tiles (32 rows, 64 columns)
    max_items += ((p->Np + 31) / 32) * ((p->Pp + 63) / 64) + ((p->Nm + 31) / 32) * ((p->Pm + 63) / 64);
  }
  {
    const char* e = getenv("PPL_BATCH_BRANCHES");
    if (e) b->n_branches = std::max(1, std::min(ppl_batch_s::kBranches, atoi(e)));
    std::vector<int> order(n);
    for (int k = 0; k < n; ++k) order[k] = k;
    auto work = [&](int k) { return build_flops(b->plans[k], 0, b->plans[k]->v); };
    std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return work(x) > work(y); });
    double load[ppl_batch_s::kBranches] = {0};
    b->branch_of.assign(n, 0);
    for (int k : order) {
      int j = 0;
      for (int q = 1; q < b->n_branches; ++q)
        if (load[q] < load[j]) j = q;
      b->branch_of[k] = j;
      load[j] += work(k);
    }
  }
  Layout L;
  L.cur = off;
  for (int j = 0; j < b->n_branches; ++j) {
    uint64_t gb = 0;
    for (int k = 0; k < n; ++k)
      if (b->branch_of[k] == j) gb = std::max<uint64_t>(gb, b->plans[k]->g_bytes_wanted);
    b->g_branch[j] = L.take(gb);
  }
  b->groups_r = L.take((uint64_t)2 * n * sizeof(GroupDesc));
  b->items_r = L.take((uint64_t)max_items * sizeof(int4));
  b->counter_r = L.take(256);
  b->max_items = max_items;
  b->need = L.cur;
  *out = b;
  return PPL_OK;
}

int ppl_batch_query(ppl_batch_t b, uint64_t* bytes, int32_t* n_items) {
  if (!b) return fail(PPL_E_ARG, "null batch");
  if (bytes) *bytes = b->need;
  if (n_items) *n_items = (int32_t)b->items.size();
  return PPL_OK;
}

int ppl_batch_bind_workspace(ppl_batch_t b, void* dptr, uint64_t bytes) {
  g_err[0] = 0;
  if (!b || !dptr) return fail(PPL_E_ARG, "null argument");
  if (((uintptr_t)dptr) % 256 != 0) return fail(PPL_E_ARG, "workspace must be 256-byte aligned");
  if (bytes < b->need) return fail(PPL_E_NOMEM, "batch workspace needs %llu bytes", (unsigned long long)b->need);
  for (int k = 0; k < b->n; ++k) {
    ppl_plan_t p = b->plans[k];
    PPL_TRY(ppl_bind_workspace(p, (char*)dptr + b->offs[k], p->ws_bytes_needed));
    // the branch's build scratch, addressed from the plan's part of the workspace
    const Region& gb = b->g_branch[b->branch_of[k]];
    p->g.off = gb.off - b->offs[k];
    p->g.bytes = gb.bytes;
  }
  b->ws = (char*)dptr;
  b->built = b->prepared = false;
  batch_drop_graph(b);
  return PPL_OK;
}

int ppl_batch_build(ppl_batch_t b, const double* const* L) {
  g_err[0] = 0;
  PPL_TRY(batch_check(b));
  if (!L) return fail(PPL_E_ARG, "null L array");
  for (int k = 0; k < b->n; ++k) {
    if (!L[k]) return fail(PPL_E_ARG, "null L for instance %d", k);
    PPL_TRY(check_symmetric(b->plans[k], L[k]));
  }
  PPL_TRY(batch_build_branches(b, L, true));
  b->built = true;
  return batch_prepare(b);
}

int ppl_batch_autotune(ppl_batch_t b, int32_t reps) {
  g_err[0] = 0;
  PPL_TRY(batch_check(b));
  if (!b->built) return fail(PPL_E_STATE, "build the batch before autotuning");
  if (reps < 1) return fail(PPL_E_ARG, "reps must be >= 1");
  batch_drop_graph(b);
  // Policies timed on the real grouped launch (operand values do not matter): the
  // model's tile for every GEMM, and for each grouped tile t, t wherever it pads the
  // occupied-pair rows by at most a quarter (the model's tile elsewhere).
  const int nt = contract_tile_count();
  std::vector<int> best_tiles(2 * b->n, -1);
  double best_ms = 1e300;
  hipEvent_t e0, e1;
  PPL_HIP_TRY(hipEventCreate(&e0));
  PPL_HIP_TRY(hipEventCreate(&e1));
  int rc = PPL_OK;
  for (int pol = -1; pol < nt && rc == PPL_OK; ++pol) {
    if (pol >= 0 && !grouped_tile_ok(pol)) continue;
    b->gtile.assign(2 * b->n, -1);
    if (pol >= 0) {
      int bm, bn;
      grouped_tile_dims(pol, &bm, &bn);
      for (int k = 0; k < b->n; ++k)
        for (int which = 0; which < 2; ++which) {
          const int64_t M = which == 0 ? b->plans[k]->Np : b->plans[k]->Nm;
          if (M > 0 && (double)M / (double)((M + bm - 1) / bm * bm) >= 0.75) b->gtile[2 * k + which] = pol;
        }
    }
    if ((rc = batch_prepare(b)) != PPL_OK) break;
    auto launch = [&]() {
      const int n_items = (int)b->items.size();
      return gemm_grouped(b->stream, b->prec, b->ws, reinterpret_cast<const GroupDesc*>(b->ws + b->groups_r.off),
                          reinterpret_cast<const int4*>(b->ws + b->items_r.off), n_items,
                          reinterpret_cast<const int*>(b->ws + b->counter_r.off + kQueueBeginOffset),
                          reinterpret_cast<int*>(b->ws + b->counter_r.off), n_items < 512 ? n_items : 512);
    };
    if ((rc = launch()) != PPL_OK) break;
    if (hipEventRecord(e0, b->stream) != hipSuccess) { rc = fail(PPL_E_HIP, "event record failed"); break; }
    for (int r = 0; r < reps && rc == PPL_OK; ++r) rc = launch();
    if (rc != PPL_OK) break;
    float ms = 0.f;
    if (hipEventRecord(e1, b->stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
        hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
      rc = fail(PPL_E_HIP, "event timing failed");
      break;
    }
    if (ms < best_ms) {
      best_ms = ms;
      best_tiles = b->gtile;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  b->gtile = best_tiles;
  const int rc2 = batch_prepare(b);
  return rc != PPL_OK ? rc : rc2;
}

int ppl_batch_contract(ppl_batch_t b, const double* const* t2, double* const* R) {
  g_err[0] = 0;
  PPL_TRY(batch_check(b));
  if (!t2 || !R) return fail(PPL_E_ARG, "null pointer array");
  if (!b->built || !b->prepared) return fail(PPL_E_STATE, "batch not built");
  return batch_enqueue(b, t2, R);
}

int ppl_batch_graph_capture(ppl_batch_t b, const double* const* t2, double* const* R) {
  g_err[0] = 0;
  PPL_TRY(batch_check(b));
  if (!t2 || !R) return fail(PPL_E_ARG, "null pointer array");
  if (!b->built || !b->prepared) return fail(PPL_E_STATE, "batch not built");
  if (b->stream == nullptr) return fail(PPL_E_ARG, "graph capture needs a non-default stream");
  batch_drop_graph(b);
  for (int k = 0; k < b->n; ++k) b->plans[k]->prof_on = false;
  PPL_HIP_TRY(hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal));
  const int rc = batch_enqueue(b, t2, R);
  hipGraph_t g = nullptr;
  const hipError_t e = hipStreamEndCapture(b->stream, &g);
  if (rc != PPL_OK) {
    if (g) (void)hipGraphDestroy(g);
    return rc;
  }
  if (e != hipSuccess) return fail(PPL_E_HIP, "hipStreamEndCapture failed: %s", hipGetErrorString(e));
  b->graph = g;
  const hipError_t e2 = hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0);
  if (e2 != hipSuccess) {
    batch_drop_graph(b);
    return fail(PPL_E_HIP, "hipGraphInstantiate failed: %s", hipGetErrorString(e2));
  }
  return PPL_OK;
}

int ppl_batch_graph_capture_build(ppl_batch_t b, const double* const* L, const double* const* t2,
                                  double* const* R) {
  g_err[0] = 0;
  PPL_TRY(batch_check(b));
  if (!L || !t2 || !R) return fail(PPL_E_ARG, "null pointer array");
  for (int k = 0; k < b->n; ++k)
    if (!L[k] || !t2[k] || !R[k]) return fail(PPL_E_ARG, "null L, t2 or R for instance %d", k);
  if (!b->built || !b->prepared) return fail(PPL_E_STATE, "build the batch once (ppl_batch_build) before capturing");
  if (b->stream == nullptr) return fail(PPL_E_ARG, "graph capture needs a non-default stream");
  batch_drop_graph(b);
  for (int k = 0; k < b->n; ++k) b->plans[k]->prof_on = false;
  PPL_HIP_TRY(hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal));
  int rc = batch_build_branches(b, L, false);
  if (rc == PPL_OK) rc = batch_enqueue(b, t2, R);
  hipGraph_t g = nullptr;
  const hipError_t e = hipStreamEndCapture(b->stream, &g);
  if (rc != PPL_OK) {
    if (g) (void)hipGraphDestroy(g);
    return rc;
  }
  if (e != hipSuccess) return fail(PPL_E_HIP, "hipStreamEndCapture failed: %s", hipGetErrorString(e));
  b->graph = g;
  const hipError_t e2 = hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0);
  if (e2 != hipSuccess) {
    batch_drop_graph(b);
    return fail(PPL_E_HIP, "hipGraphInstantiate failed: %s", hipGetErrorString(e2));
  }
  return PPL_OK;
}

int ppl_batch_graph_launch(ppl_batch_t b) {
  g_err[0] = 0;
  PPL_TRY(batch_check(b));
  if (!b->exec) return fail(PPL_E_STATE, "no captured graph");
  PPL_HIP_TRY(hipGraphLaunch(b->exec, b->stream));
  return PPL_OK;
}

int ppl_batch_destroy(ppl_batch_t b) {
  if (!b) return PPL_OK;
  batch_drop_graph(b);
  for (int j = 0; j < ppl_batch_s::kBranches; ++j) {
    if (b->side[j]) {
      (void)hipStreamSynchronize(b->side[j]);
      (void)hipStreamDestroy(b->side[j]);
    }
    if (b->ev_join[j]) (void)hipEventDestroy(b->ev_join[j]);
  }
  if (b->ev_fork) (void)hipEventDestroy(b->ev_fork);
  for (ppl_plan_t p : b->plans) ppl_destroy(p);
  delete b;
  return PPL_OK;
}

}  // extern "C"
