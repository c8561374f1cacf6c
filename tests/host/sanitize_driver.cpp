// Host-side checks run under AddressSanitizer + UndefinedBehaviorSanitizer (CPU only): the
// library's host paths -- delay tables, the beam-model SB table, argument validation of the
// entry points -- are called with valid and invalid arguments.  Prints one line per check:
//   <name> <status> [<sum of the output> <max>]
// which tests/test_host_sanitizers.py compares with the oracle and the expected statuses.
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <limits>
#include <vector>

#include "arts.h"

static void band(int nchan, double* f_lo, double* df) {
  *df = 300.0 / nchan;
  *f_lo = 1220.0 + *df / 2.0;
}

static void delay_line(const char* name, int nchan, double f_lo, double df, double tsamp,
                       const std::vector<double>& dms, int ds) {
  std::vector<int32_t> out(static_cast<size_t>(nchan) * dms.size(), -1);
  double margin = -1;
  const int st = arts_delay_table(nchan, f_lo, df, tsamp, dms.data(),
                                  static_cast<int32_t>(dms.size()), ds, out.data(), &margin);
  long long sum = 0, mx = 0;
  for (int32_t v : out) {
    sum += v;
    mx = v > mx ? v : mx;
  }
  std::printf("%s %d %lld %lld\n", name, st, sum, mx);
}

int main() {
  const double tsamp = 81.92e-6;
  double f_lo, df;
  // valid delay tables: the small case, the Apertif case, D = 4, a descending band
  band(128, &f_lo, &df);
  std::vector<double> dms;
  for (int i = 0; i < 256; ++i) dms.push_back(0.5 * i);
  delay_line("delays_small", 128, f_lo, df, tsamp, dms, 1);
  band(1536, &f_lo, &df);
  dms.clear();
  for (int i = 0; i < 2048; ++i) dms.push_back(i);
  delay_line("delays_apertif", 1536, f_lo, df, tsamp, dms, 1);
  dms.clear();
  for (int i = 0; i < 1476; ++i) dms.push_back(2048.0 + 2.0 * i);
  delay_line("delays_ds4", 1536, f_lo, df, tsamp, dms, 4);
  delay_line("delays_descending", 384, 1519.609375, -300.0 / 384, tsamp, {0.0, 10.0, 500.0}, 1);
  // invalid arguments
  const std::vector<double> one = {10.0};
  const std::vector<double> nan = {std::numeric_limits<double>::quiet_NaN()};
  const std::vector<double> neg = {-1.0};
  delay_line("bad_nchan", 0, 1220.0, 1.0, tsamp, one, 1);
  delay_line("bad_df", 16, 1220.0, 0.0, tsamp, one, 1);
  delay_line("bad_tsamp", 16, 1220.0, 1.0, -1.0, one, 1);
  delay_line("bad_dm_nan", 16, 1220.0, 1.0, tsamp, nan, 1);
  delay_line("bad_dm_neg", 16, 1220.0, 1.0, tsamp, neg, 1);
  delay_line("bad_ds", 16, 1220.0, 1.0, tsamp, one, 0);
  delay_line("bad_freq", 16, -100.0, 1.0, tsamp, one, 1);
  delay_line("bad_huge", 16, 1.0, 1.0, 1e-12, {1e9}, 1);
  std::printf("bad_null_out %d\n", arts_delay_table(16, 1220.0, 1.0, tsamp, one.data(), 1, 1,
                                                       nullptr, nullptr));
  // beam-model SB tables (71 halfway switches, 151 quarter blends)
  for (int q = 0; q < 2; ++q) {
    const int nsb = q ? 151 : 71;
    std::vector<uint8_t> tbl(static_cast<size_t>(nsb) * 1536, 255);
    double margin = -1;
    band(1536, &f_lo, &df);
    const int st = arts_sb_table_beam_model(nsb, 12, 1536, f_lo, df, 1500.0, 0.80, 1296.0,
                                            144.0, q, tbl.data(), &margin);
    long long sum = 0, mx = 0;
    for (uint8_t v : tbl) {
      sum += v;
      mx = v > mx ? v : mx;
    }
    std::printf("sb_table_%d %d %lld %lld\n", nsb, st, sum, mx);
  }
  std::vector<uint8_t> small(64);
  std::printf("sb_bad_ntab %d\n", arts_sb_table_beam_model(4, 3, 16, 1220.0, 1.0, 1500.0, 0.8,
                                                          1296.0, 144.0, 0, small.data(), nullptr));
  std::printf("sb_bad_alpha %d\n", arts_sb_table_beam_model(4, 12, 16, 1220.0, 1.0, 1500.0, -1.0,
                                                           1296.0, 144.0, 0, small.data(), nullptr));
  std::printf("sb_null %d\n", arts_sb_table_beam_model(4, 12, 16, 1220.0, 1.0, 1500.0, 0.8,
                                                      1296.0, 144.0, 0, nullptr, nullptr));
  // plan creation: argument checks come before any device call
  band(64, &f_lo, &df);
  const int32_t w_bad[] = {1, 4, 2};
  const int32_t w_ok[] = {1, 2, 4};
  arts_plan_t p = nullptr;
  std::printf("plan_bad_widths %d\n",
              arts_plan_create(64, f_lo, df, tsamp, one.data(), 1, w_bad, 3, &p));
  std::printf("plan_zero_widths %d\n",
              arts_plan_create(64, f_lo, df, tsamp, one.data(), 1, w_ok, 0, &p));
  std::printf("plan_null_out %d\n",
              arts_plan_create(64, f_lo, df, tsamp, one.data(), 1, w_ok, 3, nullptr));
  std::printf("plan_bad_dm %d\n", arts_plan_create(64, f_lo, df, tsamp, nan.data(), 1, w_ok, 3, &p));
  // calls on NULL objects are refused, never dereferenced
  int64_t n = 0;
  int32_t v = 0;
  std::printf("null_plan_candidates %d\n",
              arts_candidates(nullptr, nullptr, 1, 100, 8.0f, 0, 0, nullptr, 0, &n, nullptr));
  std::printf("null_plan_noalloc %d\n",
              arts_candidates_noalloc(nullptr, nullptr, 1, 100, 8.0f, 0, 0, nullptr, 0, &n,
                                      nullptr));
  std::printf("null_plan_tiling %d\n", arts_plan_set_tiling_shape(nullptr, 0, 1, 0));
  std::printf("null_plan_get_tiling %d\n", arts_plan_get_tiling(nullptr, &v));
  std::printf("null_stream_push %d\n", arts_stream_push(nullptr, nullptr, nullptr));
  std::printf("null_stream_wait %d\n", arts_stream_wait(nullptr, nullptr, 0, &n, nullptr));
  std::printf("null_server_tick %d\n", arts_server_tick(nullptr, nullptr));
  std::printf("null_server_poll %d\n", arts_server_poll(nullptr, 0, nullptr));
  std::printf("bad_server_budget %d\n", arts_server_create(0, nullptr));
  std::printf("null_batch_create %d\n", arts_batch_create(nullptr));
  std::printf("bad_tiling_describe %d\n", arts_tiling_describe(-1, nullptr, 0));
  for (int s = 0; s >= -8; --s) std::printf("strerror %d %s\n", s, arts_strerror(s));
  arts_stream_destroy(nullptr);
  arts_plan_destroy(nullptr);
  std::printf("done 0\n");
  return 0;
}
