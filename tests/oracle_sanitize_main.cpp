// Test driver: the oracle built with AddressSanitizer and
// UndefinedBehaviorSanitizer runs tracking (float and double, indexed and
// brute scans), the margin check, the FP64 replay, the refit with its
// gradient and the ambiguity solving on an input file written by the test.
// Any sanitizer report makes the process fail.
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "../oracle/kalman.h"

extern "C" {
void* orc_track(int precision, const float* row_x, int n_rows, const OrcParams* p, int n_units,
                const int64_t* row_begin, const float* y, const float* z, int unit_lo, int unit_hi,
                int n_threads);
void orc_free(void* h);
int64_t orc_len(void* h, const char* name);
int orc_get(void* h, const char* name, void* dst);
int64_t orc_margins(const float* row_x, int n_rows, const OrcParams* p, int n_units,
                    const int64_t* row_begin, const float* y, const float* z, double eps,
                    double eps_gap, uint8_t* flags);
void orc_replay(int precision, const float* row_x, int n_rows, const OrcParams* p, const float* y,
                const float* z, int64_t n_tracks, const int64_t* hit_begin, const int32_t* hits,
                const uint8_t* rows, const int32_t* r0, const int32_t* flags, double* param,
                double* cov, double* chi2, double* xref, int32_t* ok, double* smax);
void orc_refit(const float* row_x, const OrcParams* p, int64_t n_tracks, const int64_t* hit_begin,
               const int32_t* hit_id, const uint8_t* hit_row, const int32_t* unit,
               const float* unit_alpha, const float* seed, const float* y, const float* z,
               const double* theta, int32_t z_fixed, double z_map, double* chi2, int32_t* ok);
void orc_refit_grad(const float* row_x, const OrcParams* p, int64_t n_tracks,
                    const int64_t* hit_begin, const int32_t* hit_id, const uint8_t* hit_row,
                    const int32_t* unit, const float* unit_alpha, const float* seed, const float* y,
                    const float* z, const double* theta, const double* dL_dchi2, double* grad,
                    double* hit_grad);
int64_t orc_select(int64_t n_tracks, const int32_t* unit, const int32_t* n, const int64_t* hit_begin,
                   const int32_t* hit_id, const float* chi2, const int32_t* ndf, int64_t n_clusters,
                   int32_t shared_num, int32_t shared_den, uint8_t* keep, int32_t* assign);
int orc_map_ncoef();
void orc_fit(int precision, int decide, const float* row_x, const OrcParams* p, float chi2_cut, float vs, float vt,
             float vw, int64_t n_tracks, const int64_t* hit_begin, const int32_t* hit_id, const uint8_t* hit_row,
             const float* seed, const float* x_ref, const float* y, const float* z, uint8_t* reject, double* param,
             double* cov, double* chi2, double* x_out, int32_t* n_kept, int32_t* ok);
void orc_rebuild(int precision, const float* row_x, int n_rows, const OrcParams* p, float chi2_cut,
                 float chi2_final, float vs, float vt, float vw, int32_t k_max, int32_t rounds,
                 int32_t extrapolate, float chi2_extrap, int32_t n_units, int64_t n_tracks, const int32_t* unit, const int64_t* hit_begin, const int32_t* hit_id,
                 const uint8_t* hit_row, const float* seed, const float* x_ref, const float* t_chi2,
                 const int32_t* t_ndf, const int64_t* row_begin, const float* y, const float* z,
                 int32_t* assigned, double* param, double* cov, double* chi2_out, double* x_out,
                 int32_t* n_kept, int32_t* ok);
struct OrcMergeParams {
  float x_m, cos_h, sin_h;
  float tol[5];
  float chi2_cut;
  int32_t cross_electrode;
};
int orc_merge_views(const OrcParams* p, const OrcMergeParams* mp, int precision, int64_t n_tracks,
                    const float* param, const float* x_ref, double* views, uint8_t* ok);
int orc_merge(const OrcParams* p, const OrcMergeParams* mp, int64_t n_tracks, int32_t n_units,
              const int32_t* unit, const float* param, const float* x_ref, const int32_t* r_in,
              const int32_t* r_out, const int32_t* unit_nbr, int32_t* prev, int32_t* next, int32_t* root);
}

template <class T>
std::vector<T> get(void* h, const char* name) {
  std::vector<T> v(size_t(orc_len(h, name)));
  orc_get(h, name, v.data());
  return v;
}

int main(int argc, char** argv) {
  if (argc != 2) return 2;
  FILE* f = std::fopen(argv[1], "rb");
  if (!f) return 2;
  int32_t n_rows = 0, n_units = 0;
  int64_t n = 0;
  if (std::fread(&n_rows, 4, 1, f) != 1 || std::fread(&n_units, 4, 1, f) != 1 || std::fread(&n, 8, 1, f) != 1)
    return 2;
  std::vector<float> row_x(n_rows), y(n), z(n), alpha(n_units);
  std::vector<int64_t> rb(size_t(n_units) * n_rows + 1);
  if (std::fread(row_x.data(), 4, n_rows, f) != size_t(n_rows) ||
      std::fread(rb.data(), 8, rb.size(), f) != rb.size() || std::fread(y.data(), 4, n, f) != size_t(n) ||
      std::fread(z.data(), 4, n, f) != size_t(n) || std::fread(alpha.data(), 4, n_units, f) != size_t(n_units))
    return 2;
  std::fclose(f);
  OrcParams p{2.0f, 2.0f, 0.36f, 16.0f, 0.99f, 0.1f, 0.1f, 0.1f, 100.0f, 0.5f, 10, 8, 8, 0};
  for (int brute = 0; brute < 2; ++brute) {
    p.brute = brute;
    for (int prec : {32, 64}) orc_free(orc_track(prec, row_x.data(), n_rows, &p, n_units, rb.data(), y.data(),
                                                 z.data(), -1, -1, 2));
  }
  p.brute = 0;
  std::vector<uint8_t> flags(n, 0);
  orc_margins(row_x.data(), n_rows, &p, n_units, rb.data(), y.data(), z.data(), 1e-5, 1e-3, flags.data());
  void* h = orc_track(32, row_x.data(), n_rows, &p, n_units, rb.data(), y.data(), z.data(), -1, -1, 2);
  auto t_n = get<int32_t>(h, "t_n");
  auto t_hb = get<int64_t>(h, "t_hit_begin");
  auto t_hits = get<int32_t>(h, "t_hits");
  auto t_rows = get<uint8_t>(h, "t_rows");
  auto t_r0 = get<int32_t>(h, "t_r0");
  auto t_flags = get<int32_t>(h, "t_flags");
  auto t_unit = get<int32_t>(h, "t_unit");
  auto t_param = get<double>(h, "t_param");
  auto t_chi2 = get<double>(h, "t_chi2");
  auto t_ndf = get<int32_t>(h, "t_ndf");
  orc_free(h);
  const int64_t nt = int64_t(t_n.size());
  std::vector<double> param(5 * nt), cov(15 * nt), chi2(nt), xref(nt);
  std::vector<int32_t> ok(nt);
  std::vector<double> smax(nt);
  orc_replay(64, row_x.data(), n_rows, &p, y.data(), z.data(), nt, t_hb.data(), t_hits.data(), t_rows.data(),
             t_r0.data(), t_flags.data(), param.data(), cov.data(), chi2.data(), xref.data(), ok.data(),
             smax.data());
  std::vector<float> seed(5 * nt), fchi2(nt);
  for (int64_t i = 0; i < 5 * nt; ++i) seed[i] = float(t_param[i]);
  for (int64_t i = 0; i < nt; ++i) fchi2[i] = float(t_chi2[i]);
  const int nc = orc_map_ncoef();
  std::vector<double> theta(nc), grad(nc), w(nt, 1.0);
  for (int i = 0; i < nc; ++i) theta[i] = 0.01 * double((i * 7919) % 13 - 6);
  std::vector<double> rchi2(nt);
  std::vector<int32_t> rok(nt);
  orc_refit(row_x.data(), &p, nt, t_hb.data(), t_hits.data(), t_rows.data(), t_unit.data(), alpha.data(),
            seed.data(), y.data(), z.data(), theta.data(), 0, 0.0, rchi2.data(), rok.data());
  orc_refit(row_x.data(), &p, nt, t_hb.data(), t_hits.data(), t_rows.data(), t_unit.data(), alpha.data(),
            seed.data(), y.data(), z.data(), theta.data(), 1, 0.0, rchi2.data(), rok.data());
  const int64_t ng = nt < 40 ? nt : 40;  // the forward-mode gradient is slow: a few tracks
  orc_refit_grad(row_x.data(), &p, ng, t_hb.data(), t_hits.data(), t_rows.data(), t_unit.data(), alpha.data(),
                 seed.data(), y.data(), z.data(), theta.data(), w.data(), grad.data(), nullptr);
  std::vector<uint8_t> keep(nt);
  std::vector<int32_t> assign(n);
  const int64_t kept = orc_select(nt, t_unit.data(), t_n.data(), t_hb.data(), t_hits.data(), fchi2.data(),
                                  t_ndf.data(), n, 1, 10, keep.data(), assign.data());
  auto t_xref = std::vector<float>(nt);
  {
    void* h2 = orc_track(32, row_x.data(), n_rows, &p, n_units, rb.data(), y.data(), z.data(), -1, -1, 2);
    auto xr64 = get<double>(h2, "t_xref");
    for (int64_t i = 0; i < nt; ++i) t_xref[i] = float(xr64[i]);
    orc_free(h2);
  }
  std::vector<uint8_t> rej(t_hits.size());
  std::vector<double> fp(5 * nt), fc(15 * nt), fchi(nt), fx(nt);
  std::vector<int32_t> fk(nt), fok(nt);
  for (int prec : {32, 64})
    orc_fit(prec, prec == 32, row_x.data(), &p, 16.0f, 1e-2f, 1e-2f, 1.0f, nt, t_hb.data(), t_hits.data(),
            t_rows.data(), seed.data(), t_xref.data(), y.data(), z.data(), rej.data(), fp.data(), fc.data(),
            fchi.data(), fx.data(), fk.data(), fok.data());
  std::vector<int32_t> assigned(size_t(nt) * n_rows);
  for (int prec : {32, 64})
    for (int ex : {0, 1})
    orc_rebuild(prec, row_x.data(), n_rows, &p, 16.0f, 16.0f, 1e-2f, 1e-2f, 1.0f, 4, 6, ex, 9.0f, n_units, nt,
                t_unit.data(),
                t_hb.data(), t_hits.data(), t_rows.data(), seed.data(), t_xref.data(), fchi2.data(), t_ndf.data(),
                rb.data(), y.data(), z.data(), assigned.data(), fp.data(), fc.data(), fchi.data(), fx.data(),
                fk.data(), fok.data());
  {
    // merging of the tracklets (units = sectors 0 .. n_units - 1 of one half)
    const OrcMergeParams mp{165.0f, 0.98480775f, 0.17364818f, {1.0f, 1.0f, 0.02f, 0.02f, 0.1f}, 25.0f, 1};
    std::vector<int32_t> r_in(nt), r_out(nt), nbr(size_t(3) * n_units), prv(nt), nxt(nt), root(nt);
    for (int64_t i = 0; i < nt; ++i) {
      r_in[i] = t_rows[size_t(t_hb[i])];
      r_out[i] = t_rows[size_t(t_hb[i + 1] - 1)];
    }
    for (int u = 0; u < n_units; ++u) {
      nbr[3 * u + 0] = u + 1 < n_units ? u + 1 : -1;
      nbr[3 * u + 1] = u > 0 ? u - 1 : -1;
      nbr[3 * u + 2] = -1;
    }
    std::vector<double> views(size_t(15) * nt);
    std::vector<uint8_t> vok(size_t(3) * nt);
    for (int prec : {32, 64})
      orc_merge_views(&p, &mp, prec, nt, seed.data(), t_xref.data(), views.data(), vok.data());
    orc_merge(&p, &mp, nt, n_units, t_unit.data(), seed.data(), t_xref.data(), r_in.data(), r_out.data(),
              nbr.data(), prv.data(), nxt.data(), root.data());
  }
  std::printf("tracklets %lld kept %lld\n", static_cast<long long>(nt), static_cast<long long>(kept));
  return 0;
}
