// Host-side checks of libppl, built with AddressSanitizer and UndefinedBehaviorSanitizer on
// the host code (tests/test_host_sanitizers.py builds and runs it on the CPU; no GPU is
// used): the planner over many shapes, precisions, budgets and flags, the tune-cache parser
// on malformed files, the batched and MLP handles, argument and state errors of the device
// entry points (which must fail before touching a device), the DIIS subspace solve on
// well-posed, singular and malformed systems, and the tile plans and cube packing of the
// upper-triangle build.
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#include <unistd.h>

#include <cmath>
#include <random>
#include <string>
#include <vector>

#include "diis_solve.h"
#include "pack_cubes.h"
#include "ppl.h"

namespace ppl {   // host-side build planning of the library (not part of the C ABI)
int build_tile_dims(int tile, int* bm, int* bn);
void build_tile_table_sym(int tile, int v, int a0, int a1, std::vector<int>& tiles, int& n_mtiles, int& n_ntiles);
void build_column_order(int v, std::vector<int>& cols);
}  // namespace ppl

static int failures = 0;
static int checks = 0;
#define CHECK(cond)                                                                  \
  do {                                                                               \
    ++checks;                                                                        \
    if (!(cond)) {                                                                   \
      fprintf(stderr, "CHECK failed at %s:%d: %s (%s)\n", __FILE__, __LINE__, #cond, \
              ppl_last_error());                                                     \
      ++failures;                                                                    \
    }                                                                                \
  } while (0)

static ppl_desc_t make_desc(int o, int v, int naux, int prec, uint64_t budget) {
  ppl_desc_t d;
  memset(&d, 0, sizeof(d));
  d.o = o;
  d.v = v;
  d.naux = naux;
  d.prec = prec;
  d.tile_contract = -1;
  d.hbm_budget = budget;
  return d;
}

static void check_planner() {
  const int shapes[][3] = {{1, 2, 1},    {3, 17, 23},   {5, 20, 60},   {20, 200, 600}, {40, 400, 1200},
                           {100, 700, 4000}, {7, 33, 5}, {1, 300, 2},   {30, 300, 900}, {2, 3, 70000}};
  const uint64_t budgets[] = {1ull << 42, 64ull << 30, 2ull << 30, 64ull << 20, 1ull << 20};
  for (const auto& sh : shapes)
    for (int prec = 0; prec < 4; ++prec)
      for (uint64_t budget : budgets)
        for (int flags = 0; flags < 3; ++flags)
          for (int keep = 0; keep < 2; ++keep) {
            ppl_desc_t d = make_desc(sh[0], sh[1], sh[2], prec, budget);
            d.flags = flags;
            d.keep_fp64 = keep;
            d.diis_max = flags == 0 ? 8 : 0;
            d.build_scratch = flags == 2 ? (256ull << 20) : 0;
            ppl_plan_t p = nullptr;
            const int rc = ppl_plan(&d, &p);
            CHECK(rc == PPL_OK || rc == PPL_E_NOMEM);
            if (rc != PPL_OK) {
              CHECK(p == nullptr);
              continue;
            }
            ppl_plan_info_t info;
            CHECK(ppl_plan_query(p, &info) == PPL_OK);
            const int64_t v = sh[1], o = sh[0];
            CHECK(info.p_plus == v * (v + 1) / 2 && info.p_minus == v * (v - 1) / 2);
            CHECK(info.n_plus == o * (o + 1) / 2 && info.n_minus == o * (o - 1) / 2);
            CHECK(info.workspace_bytes <= budget);
            CHECK(info.n_batches >= 1);
            CHECK(info.resident == 0 || info.resident == 1);
            CHECK(info.tile_contract >= 0 && info.tile_contract < ppl_tile_count());
            CHECK(info.splits_contract >= 0 && info.splits_contract <= 8);
            const double pp = (double)info.p_plus, pm = (double)info.p_minus;
            CHECK(info.flops_contract == 2.0 * (pp * pp * info.n_plus + pm * pm * info.n_minus));
            CHECK(ppl_destroy(p) == PPL_OK);
          }
  // argument errors
  const int bad[][3] = {{0, 10, 5}, {2, 1, 5}, {2, 10, 0}, {2, 40000, 5}, {-3, 10, 5}};
  for (const auto& b : bad) {
    ppl_desc_t d = make_desc(b[0], b[1], b[2], PPL_FP64, 1ull << 30);
    ppl_plan_t p = nullptr;
    CHECK(ppl_plan(&d, &p) == PPL_E_ARG && p == nullptr);
  }
  {
    ppl_desc_t d = make_desc(3, 8, 6, 9, 1ull << 30);
    ppl_plan_t p = nullptr;
    CHECK(ppl_plan(&d, &p) == PPL_E_ARG);
    d.prec = PPL_FP64;
    d.tile_contract = 99;
    CHECK(ppl_plan(&d, &p) == PPL_E_ARG);
    d.tile_contract = -1;
    d.diis_max = PPL_DIIS_MAX + 1;
    CHECK(ppl_plan(&d, &p) == PPL_E_ARG);
    d.diis_max = 0;
    d.flags = 8;
    CHECK(ppl_plan(&d, &p) == PPL_E_ARG);
    d.flags = PPL_PLAN_CONTRACT_ONLY | PPL_PLAN_RING;
    CHECK(ppl_plan(&d, &p) == PPL_E_ARG);
    CHECK(ppl_plan(nullptr, &p) == PPL_E_ARG);
    CHECK(ppl_plan(&d, nullptr) == PPL_E_ARG);
    // hbm_budget 0 asks the device: without one, a HIP error (not a crash)
    d = make_desc(3, 8, 6, PPL_FP64, 0);
    const int rc = ppl_plan(&d, &p);
    CHECK(rc == PPL_OK || rc == PPL_E_HIP);
    if (rc == PPL_OK) ppl_destroy(p);
  }
}

static std::string write_file(const std::string& text) {
  char path[] = "/tmp/ppl_tune_XXXXXX";
  const int fd = mkstemp(path);
  CHECK(fd >= 0);
  if (fd < 0) return "";
  const ssize_t n = write(fd, text.data(), text.size());
  CHECK(n == (ssize_t)text.size());
  close(fd);
  return path;
}

static void plan_config(const char* cache, int prec, int o, int v, int naux, int cfg[4]) {
  ppl_desc_t d = make_desc(o, v, naux, prec, 1ull << 42);
  d.tune_cache = cache;
  ppl_plan_t p = nullptr;
  CHECK(ppl_plan(&d, &p) == PPL_OK);
  ppl_plan_info_t info;
  ppl_plan_query(p, &info);
  cfg[0] = info.tile_contract;
  cfg[1] = info.splits_contract;
  cfg[2] = info.tile_contract_minus;
  cfg[3] = info.splits_contract_minus;
  ppl_destroy(p);
}

static void check_tune_cache() {
  std::string text = "ppl-tune 1 0 20 200 5 3 7 2\n";
  text += std::string(1000, 'x') + "\n";                                    // longer than a read buffer
  text += "ppl-tune 1 0 20 200 " + std::string(600, '9') + " 1 1 1\n";       // number out of range
  text += "ppl-tune 1 0 20 200 6 0 8 6\n";                                   // the last valid entry
  text += "ppl-tune 1 0 20 200 -4 1 0 1\nppl-tune 1 0 20 200 1 99 0 1\nppl-tune 1 0\n";
  text += std::string("\x00\xff\x01ppl-tune", 11) + "\n";
  text += "ppl-tune 1 3 40 400 9 0 9 8\nppl-tune 1 3 40 400 9 7 9 8\nppl-tune 1 3 40 400 9 8 9 2\n";
  text += "ppl-tune 1 0 20 200 2 2 2";                                      // no newline at the end
  const std::string path = write_file(text);
  int cfg[4];
  plan_config(path.c_str(), PPL_FP64, 20, 200, 600, cfg);
  CHECK(cfg[0] == 6 && cfg[1] == 0 && cfg[2] == 8 && cfg[3] == 6);
  plan_config(path.c_str(), PPL_BF16X6, 40, 400, 1200, cfg);
  CHECK(cfg[0] == 9 && cfg[1] == 7 && cfg[2] == 9 && cfg[3] == 8);
  int base[4];
  plan_config(nullptr, PPL_FP32, 20, 200, 600, base);
  plan_config(path.c_str(), PPL_FP32, 20, 200, 600, cfg);
  CHECK(memcmp(cfg, base, sizeof(cfg)) == 0);
  plan_config("/nonexistent/dir/tune.txt", PPL_FP64, 20, 200, 600, cfg);
  plan_config("/tmp", PPL_FP64, 20, 200, 600, cfg);                        // a directory: no entry
  unlink(path.c_str());
}

static void check_batch_and_mlp() {
  const int shapes[][2] = {{20, 231}, {22, 162}, {9, 101}, {24, 93}, {1, 5}, {3, 2}};
  std::vector<ppl_desc_t> d;
  for (const auto& s : shapes) d.push_back(make_desc(s[0], s[1], 3 * s[1], PPL_FP64, 0));
  ppl_batch_t b = nullptr;
  CHECK(ppl_batch_plan((int)d.size(), d.data(), &b) == PPL_OK);
  uint64_t bytes = 0;
  int32_t items = -1;
  CHECK(ppl_batch_query(b, &bytes, &items) == PPL_OK && bytes > 0 && items == 0);
  CHECK(ppl_batch_build(b, nullptr) == PPL_E_STATE);          // no workspace bound yet
  CHECK(ppl_batch_graph_launch(b) == PPL_E_STATE);
  CHECK(ppl_batch_bind_workspace(b, (void*)(uintptr_t)100, bytes) == PPL_E_ARG);   // misaligned
  CHECK(ppl_batch_destroy(b) == PPL_OK);
  CHECK(ppl_batch_plan(0, d.data(), &b) == PPL_E_ARG);
  d[1].prec = PPL_FP32;
  CHECK(ppl_batch_plan((int)d.size(), d.data(), &b) == PPL_E_ARG);
  for (auto& x : d) x.prec = PPL_BF16X3;
  CHECK(ppl_batch_plan((int)d.size(), d.data(), &b) == PPL_E_UNSUPPORTED);
  CHECK(ppl_batch_destroy(nullptr) == PPL_OK);

  ppl_mlp_t m = nullptr;
  CHECK(ppl_mlp_create(128, 4096, nullptr, &m) == PPL_OK);
  CHECK(ppl_mlp_param_count(m) == 128 * 4 + 128 + 128 * 128 + 128 + 128 + 1);
  uint64_t mb = 0;
  CHECK(ppl_mlp_workspace_bytes(m, &mb) == PPL_OK && mb > 0);
  CHECK(ppl_mlp_init(m, 1) == PPL_E_STATE);                    // no workspace bound
  std::vector<float> params(ppl_mlp_param_count(m));
  CHECK(ppl_mlp_set_params(m, params.data(), (int64_t)params.size() + 1) != PPL_OK);
  CHECK(ppl_mlp_destroy(m) == PPL_OK);
  CHECK(ppl_mlp_create(64, 4096, nullptr, &m) == PPL_E_UNSUPPORTED);
  CHECK(ppl_mlp_destroy(nullptr) == PPL_OK);
}

static void check_device_entry_errors() {
  ppl_desc_t d = make_desc(3, 8, 6, PPL_FP64, 1ull << 30);
  ppl_plan_t p = nullptr;
  CHECK(ppl_plan(&d, &p) == PPL_OK);
  void* const dev = (void*)(uintptr_t)4096;        // never dereferenced: every call fails first
  CHECK(ppl_bind_workspace(p, nullptr, 1 << 20) == PPL_E_ARG);
  CHECK(ppl_bind_workspace(p, (void*)(uintptr_t)300, 1ull << 30) == PPL_E_ARG);
  CHECK(ppl_build_batch(p, (const double*)dev, -1) == PPL_E_STATE);
  CHECK(ppl_contract(p, (const double*)dev, (double*)dev, 1.0, 0.0) == PPL_E_STATE);
  CHECK(ppl_contract_tau(p, (const double*)dev, (const double*)dev, (double*)dev, 1.0, 0.0) == PPL_E_STATE);
  CHECK(ppl_hhl(p, (const double*)dev, (const double*)dev, (double*)dev, 1.0, 0.0) == PPL_E_STATE);
  ppl_iter_opts_t o;
  ppl_iter_opts_default(&o);
  CHECK(o.max_sweeps == 100 && o.tol == 1e-7 && o.diis == 0);
  ppl_iter_report_t rep;
  CHECK(ppl_iterate(p, (const double*)dev, (const double*)dev, (const double*)dev, (double*)dev, &o, &rep) ==
        PPL_E_STATE);
  CHECK(ppl_set_contract_config(p, 99, 1, 0, 1) == PPL_E_ARG);
  CHECK(ppl_set_contract_config(p, 0, 9, 0, 1) == PPL_E_ARG);
  CHECK(ppl_autotune(p, 1, nullptr) != PPL_OK);
  CHECK(ppl_destroy(p) == PPL_OK);
  CHECK(ppl_destroy(nullptr) == PPL_OK);
  CHECK(ppl_ring(2, 4, 5, nullptr, nullptr, nullptr, 1.0, 0.0, nullptr, 0, nullptr) == PPL_E_ARG);
  CHECK(ppl_ring_static(0, 4, 5, nullptr, nullptr, nullptr, 1.0, 0.0, nullptr) == PPL_E_ARG);
  CHECK(ppl_ring_static(2, 4, 5, nullptr, nullptr, nullptr, 1.0, 0.0, nullptr) == PPL_E_ARG);
  CHECK(ppl_ring_scratch_bytes(0, 4, 5) == 0 && ppl_ring_scratch_bytes(2, 4, 0) == 0);
  CHECK(ppl_ring_scratch_bytes(32767, 32767, 1 << 30) == 0);    // byte counts overflow: no size
  CHECK(ppl_ring_scratch_bytes(10, 100, 300) > 0);
  int32_t bm, bn, th;
  for (int t = 0; t < ppl_tile_count(); ++t) CHECK(ppl_tile_dims(t, &bm, &bn, &th) == PPL_OK && bm > 0);
  CHECK(ppl_tile_dims(-1, &bm, &bn, &th) == PPL_E_ARG && ppl_tile_dims(ppl_tile_count(), &bm, &bn, &th) == PPL_E_ARG);
  CHECK(ppl_tile_dims(0, nullptr, &bn, &th) == PPL_E_ARG);
  CHECK(strlen(ppl_version()) > 0);
}

// DIIS: Gram matrices of random error vectors; the coefficients sum to one and make every
// component of B c equal (the Lagrange multiplier); degenerate and malformed systems fail.
static void check_diis() {
  constexpr int CAP = 16;
  std::mt19937_64 rng(7);
  std::normal_distribution<double> g(0.0, 1.0);
  for (int n = 1; n <= CAP; ++n)
    for (int trial = 0; trial < 4; ++trial) {
      const int dim = 40;
      std::vector<std::vector<double>> e(CAP, std::vector<double>(dim));
      for (auto& x : e)
        for (double& y : x) y = g(rng) * std::pow(0.5, trial);
      double B[CAP][CAP] = {};
      for (int i = 0; i < CAP; ++i)
        for (int j = 0; j < CAP; ++j) {
          double s = 0.0;
          for (int k = 0; k < dim; ++k) s += e[i][k] * e[j][k];
          B[i][j] = s;
        }
      std::vector<int> ids;
      for (int i = 0; i < n; ++i) ids.push_back((i * 5 + trial) % CAP);
      double c[CAP];
      CHECK(ppl::diis_solve(B, ids, c));
      double sum = 0.0;
      for (int i = 0; i < n; ++i) sum += c[i];
      CHECK(std::fabs(sum - 1.0) < 1e-10);
      double lo = 1e300, hi = -1e300;
      for (int i = 0; i < n; ++i) {
        double r = 0.0;
        for (int j = 0; j < n; ++j) r += B[ids[i]][ids[j]] * c[j];
        lo = std::min(lo, r);
        hi = std::max(hi, r);
      }
      CHECK(hi - lo <= 1e-8 * std::max(1.0, std::fabs(hi)));
    }
  double B[CAP][CAP] = {};
  double c[CAP];
  CHECK(!ppl::diis_solve(B, {0, 1}, c));                    // all zero
  for (int i = 0; i < CAP; ++i)
    for (int j = 0; j < CAP; ++j) B[i][j] = 1.0;            // identical error vectors: singular
  CHECK(!ppl::diis_solve(B, {0, 1, 2}, c));
  CHECK(ppl::diis_solve(B, {3}, c) && c[0] == 1.0);         // one vector: its own amplitudes
  B[2][2] = NAN;
  CHECK(!ppl::diis_solve(B, {2, 3}, c));
  CHECK(!ppl::diis_solve(B, {}, c));
  CHECK(!ppl::diis_solve(B, {0, CAP}, c));
  CHECK(!ppl::diis_solve(B, {-1}, c));
  std::vector<int> too_many(CAP + 1, 0);
  CHECK(!ppl::diis_solve(B, too_many, c));
}

// Upper-triangle build plan of one step: replaying the epilogue over every listed tile
// (rows the packed pairs (a, c >= a) of a in [a0, a1), columns the packed pairs (b <= d)
// from b = a0 on, products kept for b >= a, each written to G_ab[c][d] and G_ad[c][b])
// must write every entry G_ab[c][d] with b, c, d >= a exactly once, and no tile twice.
static void check_build_tables() {
  const int tiles[] = {0, 1, 5, 8, 9, 10};
  for (int v : {1, 2, 7, 40, 75})
    for (int tile : tiles)
      for (int nsteps : {1, 3}) {
        std::vector<int> cols;
        ppl::build_column_order(v, cols);
        CHECK((int64_t)cols.size() == (int64_t)v * (v + 1) / 2);
        int bm = 0, bn = 0;
        CHECK(ppl::build_tile_dims(tile, &bm, &bn) == PPL_OK);
        auto pp = [&](int64_t a, int64_t b) { return a * v - a * (a + 1) / 2 + b; };
        for (int k = 0; k < nsteps; ++k) {
          const int a0 = v * k / nsteps, a1 = v * (k + 1) / nsteps;
          if (a0 == a1) continue;
          const int W = v - a0;
          const int64_t pr0 = pp(a0, a0), pr1 = a1 >= v ? (int64_t)v * (v + 1) / 2 : pp(a1, a1);
          const int64_t M = pr1 - pr0, N = (int64_t)W * (W + 1) / 2;
          std::vector<int> list;
          int nmt = 0, nnt = 0;
          ppl::build_tile_table_sym(tile, v, a0, a1, list, nmt, nnt);
          CHECK(nmt == (int)((M + bm - 1) / bm) && nnt == (int)((N + bn - 1) / bn));
          std::vector<int> rows_a(M), rows_c(M);
          for (int a = 0, m = 0; a < v; ++a)
            for (int c = a; c < v; ++c, ++m)
              if (m >= pr0 && m < pr1) { rows_a[m - pr0] = a; rows_c[m - pr0] = c; }
          std::vector<char> seen((size_t)nmt * nnt, 0);
          std::vector<int> hits((size_t)M * W * W, 0);   // G[pair(a,b) - pr0][c - a0][d - a0]
          bool in_range = true, once = true;
          for (size_t q = 0; q + 1 < list.size(); q += 2) {
            const int mt = list[q], nt = list[q + 1];
            if (mt < 0 || mt >= nmt || nt < 0 || nt >= nnt) { in_range = false; continue; }
            if (seen[(size_t)mt * nnt + nt]++) once = false;
            for (int64_t m = (int64_t)mt * bm; m < std::min<int64_t>(M, (int64_t)(mt + 1) * bm); ++m)
              for (int64_t n = (int64_t)nt * bn; n < std::min<int64_t>(N, (int64_t)(nt + 1) * bn); ++n) {
                const int a = rows_a[m], c = rows_c[m];
                const int bd = cols[pp(a0, a0) + n], b = bd / v, d = bd % v;
                if (b < a) continue;
                hits[((size_t)(pp(a, b) - pr0) * W + (c - a0)) * W + (d - a0)]++;
                if (d != b) hits[((size_t)(pp(a, d) - pr0) * W + (c - a0)) * W + (b - a0)]++;
              }
          }
          CHECK(in_range && once);
          bool exact = true;
          for (int a = a0; a < a1; ++a)
            for (int b = a; b < v; ++b)
              for (int c = a; c < v; ++c)
                for (int d = a; d < v; ++d)
                  if (hits[((size_t)(pp(a, b) - pr0) * W + (c - a0)) * W + (d - a0)] != 1) exact = false;
          CHECK(exact);
        }
      }
}

// Cube packing of resident builds (pack_vpm_cubes_kernel): replaying its cube decode, its
// staging reads of T and the conditions of its two write passes over all steps of a
// partition must read only computed entries of T (row (a, r) of the step, column pair
// (x <= y) with x >= a), hand every cube to exactly one workgroup, write every entry of
// V+ and V- exactly once from the two integrals of its definition ((ac|bd) and (ad|bc) for
// the entry of pairs (ab), (cd), either order), and zero the padding of every row once.
static void check_pack_cubes() {
  for (int v : {1, 2, 5, 16, 17, 40, 75})
    for (int nsteps : {1, 3}) {
      const int C = ppl::kCube;
      auto pp = [&](int64_t a, int64_t b) { return a * v - a * (a + 1) / 2 + b; };
      auto pm = [&](int64_t a, int64_t b) { return a * (v - 1) - a * (a + 1) / 2 + b - 1; };
      const int64_t Pp = (int64_t)v * (v + 1) / 2, Pm = (int64_t)v * (v - 1) / 2;
      std::vector<int> pfirst(Pp), psecond(Pp);
      for (int x = 0; x < v; ++x)
        for (int y = x; y < v; ++y) { pfirst[pp(x, y)] = x; psecond[pp(x, y)] = y; }
      // the integral (pq|rs) up to its symmetries, as one number
      auto key = [&](int64_t p, int64_t q, int64_t r, int64_t t) {
        int64_t u = std::min(p, q) * v + std::max(p, q), w = std::min(r, t) * v + std::max(r, t);
        return std::min(u, w) * v * v + std::max(u, w);
      };
      std::vector<int64_t> off(v + 1, 0);
      for (int a = 0; a < v; ++a) off[a + 1] = off[a] + ppl::cubes_of(v, a);
      std::vector<int> hp((size_t)(Pp * Pp), 0), hm((size_t)(Pm * Pm), 0), padp(Pp, 0), padm(Pm, 0);
      bool reads_ok = true, values_ok = true, cubes_ok = true;
      for (int k = 0; k < nsteps; ++k) {
        const int a0 = v * k / nsteps, a1 = v * (k + 1) / nsteps;
        if (a0 == a1) continue;
        const int64_t pr0 = pp(a0, a0), W = v - a0, ldt = W * (W + 1) / 2;
        const int64_t M = (a1 >= v ? Pp : pp(a1, a1)) - pr0;
        int64_t g0 = 0, n = 0;
        for (int a = 0; a < a1; ++a) (a < a0 ? g0 : n) += ppl::cubes_of(v, a);
        CHECK(g0 == off[a0] && n == off[a1] - off[a0]);
        std::vector<int> seen((size_t)n, 0);
        std::vector<int64_t> s1((size_t)C * C * C), s2((size_t)C * C * C);
        for (int64_t bid = 0; bid < n; ++bid) {
          const int64_t g = g0 + ppl::cube_of_slot(bid, n);
          if (g < g0 || g >= g0 + n) { cubes_ok = false; continue; }
          seen[(size_t)(g - g0)]++;
          const int a = ppl::cube_virtual(off.data(), a0, a1, g);
          if (a < a0 || a >= a1 || g < off[a] || g >= off[a + 1]) { cubes_ok = false; continue; }
          const int nt = ppl::cube_blocks(v, a);
          int bi = -1, ci = -1, di = -1;
          ppl::cube_decode(g - off[a], nt, bi, ci, di);
          if (bi < 0 || bi >= nt || ci < 0 || ci > di || di >= nt) { cubes_ok = false; continue; }
          const int b0 = a + C * bi, c0 = a + C * ci, d0 = a + C * di;
          // staging as the kernel addresses T; each slot keeps the integral that address holds
          auto load = [&](std::vector<int64_t>& st, int r0, int y0) {
            for (int rl = 0; rl < C; ++rl)
              for (int bl = 0; bl < C; ++bl)
                for (int yl = 0; yl < C; ++yl) {
                  const int r = r0 + rl, b = b0 + bl, y = y0 + yl;
                  int64_t kx = -1;
                  if (r < v && b < v && y < v) {
                    const int lo = b < y ? b : y, hi = b < y ? y : b;
                    const int64_t m = pp(a, r) - pr0, col = pp(lo, hi) - pr0;
                    if (m < 0 || m >= M || col < 0 || col >= ldt) { reads_ok = false; continue; }
                    const int ra = pfirst[m + pr0], rr = psecond[m + pr0];
                    const int x = pfirst[col + pr0], x2 = psecond[col + pr0];
                    if (ra < a0 || ra >= a1 || x < ra) reads_ok = false;   // not computed by the build
                    kx = key(ra, rr, x, x2);
                  }
                  st[((size_t)rl * C + bl) * C + yl] = kx;
                }
          };
          load(s1, c0, d0);
          if (ci != di) load(s2, d0, c0);
          const std::vector<int64_t>& t2 = ci != di ? s2 : s1;
          for (int bl = 0; bl < C; ++bl)
            for (int cl = 0; cl < C; ++cl)
              for (int dl = 0; dl < C; ++dl) {
                const int b = b0 + bl, c = c0 + cl, d = d0 + dl;
                if (b >= v || d >= v || c > d) continue;
                const int64_t gcd = s1[((size_t)cl * C + bl) * C + dl], gdc = t2[((size_t)dl * C + bl) * C + cl];
                if (gcd != key(a, c, b, d) || gdc != key(a, d, b, c)) values_ok = false;
                if (!(c == a && d < b)) {                         // row (ab), column (cd) >= (ab)
                  hp[(size_t)(pp(a, b) * Pp + pp(c, d))]++;
                  if (a < b && c < d) hm[(size_t)(pm(a, b) * Pm + pm(c, d))]++;
                }
                if (!(c == a && d <= b)) {                        // the mirror entry
                  hp[(size_t)(pp(c, d) * Pp + pp(a, b))]++;
                  if (a < b && c < d) hm[(size_t)(pm(c, d) * Pm + pm(a, b))]++;
                }
              }
          if (ci == 0 && di == 0)
            for (int bl = 0; bl < C; ++bl) {
              const int b = b0 + bl;
              if (b >= v) continue;
              padp[pp(a, b)]++;
              if (a < b) padm[pm(a, b)]++;
            }
        }
        for (int x : seen) cubes_ok = cubes_ok && x == 1;
      }
      CHECK(cubes_ok && reads_ok && values_ok);
      bool once = true;
      for (int x : hp) once = once && x == 1;
      for (int x : hm) once = once && x == 1;
      for (int x : padp) once = once && x == 1;
      for (int x : padm) once = once && x == 1;
      CHECK(once);
    }
}

int main() {
  check_pack_cubes();
  check_build_tables();
  check_planner();
  check_tune_cache();
  check_batch_and_mlp();
  check_device_entry_errors();
  check_diis();
  printf("host checks: %d of %d failed\n", failures, checks);
  return failures ? 1 : 0;
}
