// The C ABI of libehi (declared in include/ehi.h): descriptor validation,
// workspace layout, state machine and the launch sequence of each stage.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <initializer_list>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "ehi_internal.h"

namespace {

thread_local std::string g_err;

ehi_status fail(ehi_status st, const std::string& msg) {
  g_err = msg;
  return st;
}

ehi_status hip_fail(hipError_t e, const char* what) {
  g_err = std::string(what) + ": " + hipGetErrorName(e) + " (" + hipGetErrorString(e) + ")";
  return EHI_EHIP;
}

#define EHI_TRY(call, what)                        \
  do {                                             \
    hipError_t e_ = (call);                        \
    if (e_ != hipSuccess) return hip_fail(e_, what); \
  } while (0)

// Resampling filter design (host, FP64): Kaiser-windowed sinc with 120 dB of
// attenuation, passband up to f_max, stopband from fs/D - f_max, cutoff
// fs/(2D); beta = 0.1102 (A - 8.7), order (A - 7.95) / (14.36 df/fs).
constexpr double kDecimAtten = 120.0;

double max_freq(const ehi_survey_desc* d) {
  double m = 0.0;
  for (int f = 0; f < d->nf; ++f) m = std::max(m, d->freq_hz[f]);
  return m;
}

// half-length K, or -1 if the stopband would start below the passband
int decim_half_length(int D, double dt, double fmax) {
  const double df_fs = 1.0 / D - 2.0 * fmax * dt;  // (fs/D - 2 f_max) / fs
  if (!(df_fs > 0)) return -1;
  const double order = (kDecimAtten - 7.95) / (14.36 * df_fs);
  return (int)std::ceil(order / 2.0);
}

// modified Bessel function of the first kind, order 0, by its power series
double bessel_i0(double x) {
  double sum = 1.0, term = 1.0;
  const double q = 0.25 * x * x;
  for (int k = 1; k < 500; ++k) {
    term *= q / ((double)k * k);
    sum += term;
    if (term < 1e-17 * sum) break;
  }
  return sum;
}

std::vector<double> decim_taps(int D, int K) {
  const double beta = 0.1102 * (kDecimAtten - 8.7);
  const double pi = 3.14159265358979323846;
  std::vector<double> h(2 * K + 1);
  double sum = 0.0;
  for (int j = -K; j <= K; ++j) {
    const double x = (double)j / D;
    const double sinc = j == 0 ? 1.0 : std::sin(pi * x) / (pi * x);
    const double r = (double)j / K;
    const double w = bessel_i0(beta * std::sqrt(std::max(0.0, 1.0 - r * r))) / bessel_i0(beta);
    h[j + K] = sinc / D * w;
    sum += h[j + K];
  }
  for (double& v : h) v /= sum;
  return h;
}

bool validate(const ehi_survey_desc* d, std::string* why) {
  auto bad = [&](const char* m) {
    *why = m;
    return false;
  };
  if (!d) return bad("descriptor is NULL");
  if (d->nz < 4 || d->nx < 4) return bad("nz and nx must be >= 4");
  if (d->nb < 0 || d->nb > ehi::kMaxSponge) return bad("nb must be in [0, 512]");
  if (!(d->h > 0) || !std::isfinite(d->h)) return bad("h must be positive and finite");
  if (!(d->dt > 0) || !std::isfinite(d->dt)) return bad("dt must be positive and finite");
  if (d->nt < 1) return bad("nt must be >= 1");
  if (d->stride != 1 && d->stride != 2 && d->stride != 4 && d->stride != 8)
    return bad("stride must be 1, 2, 4 or 8");
  if (d->nr < 1 || d->nr > 1024) return bad("nr must be in [1, 1024]");
  if (!d->rec_iz || !d->rec_ix) return bad("receiver arrays are NULL");
  for (int r = 0; r < d->nr; ++r) {
    if (d->rec_iz[r] < 0 || d->rec_iz[r] >= d->nz || d->rec_ix[r] < 0 || d->rec_ix[r] >= d->nx)
      return bad("receiver outside the interior grid");
  }
  if (d->nf < 1 || d->nf > 64) return bad("nf must be in [1, 64]");
  if (!d->freq_hz) return bad("frequency array is NULL");
  for (int f = 0; f < d->nf; ++f)
    if (!(d->freq_hz[f] >= 0) || !std::isfinite(d->freq_hz[f])) return bad("frequencies must be finite and >= 0");
  if (d->precision != EHI_PREC_PLAIN_FP32 && d->precision != EHI_PREC_SPLIT_BF16)
    return bad("unknown precision mode");
  if (d->max_ns < 1 || d->max_ns > (1 << 20)) return bad("max_ns must be in [1, 2^20]");
  if (d->nr_batch < 0) return bad("nr_batch must be >= 0");
  if (d->weighting != EHI_WEIGHT_LONG_RECORD && d->weighting != EHI_WEIGHT_FINITE_RECORD)
    return bad("unknown weighting");
  if (d->weighting == EHI_WEIGHT_FINITE_RECORD) {
    if (d->precision != EHI_PREC_SPLIT_BF16) return bad("the finite-record weighting needs the split-BF16 form");
    if (d->nr_batch != 0 && d->nr_batch < d->nr)
      return bad("the finite-record weighting needs all receivers stepped together");
  }
  long long Z = (long long)d->nz + 2LL * d->nb, X = (long long)d->nx + 2LL * d->nb;
  // buffer resources address one plane / one staging block with 31-bit byte offsets
  if ((Z + 4) * (X + 4 + ehi::kRowAlign) > (1LL << 28)) return bad("grid too large");
  long long nsub = (long long)((d->nz + d->stride - 1) / d->stride) * ((d->nx + d->stride - 1) / d->stride);
  if (d->chunk != 0 && d->chunk != 256 && d->chunk != 512 && d->chunk != 1024)
    return bad("chunk must be 0, 256, 512 or 1024");
  {
    const int nzs = (d->nz + d->stride - 1) / d->stride, nxs = (d->nx + d->stride - 1) / d->stride;
    if ((d->keep_z == 0) != (d->keep_x == 0)) return bad("keep_z and keep_x must both be 0 or both positive");
    if (d->keep_z < 0 || d->keep_z > nzs || d->keep_x < 0 || d->keep_x > nxs)
      return bad("keep_z / keep_x must be within the subgrid (0 = no compression)");
    if (d->keep_z > 0 && d->weighting == EHI_WEIGHT_FINITE_RECORD)
      return bad("spatial compression applies to the final-spectrum contraction only");
  }
  if (d->windows < 0 || d->windows > 2) return bad("windows must be 0, 1 or 2");
  if (d->herk_split < 0 || d->herk_split > ehi::kHerkSplitMax) return bad("herk_split must be in [0, 64]");
  if (d->herk_form < 0 || d->herk_form > 3) return bad("herk_form must be 0, 1, 2 or 3");
  if (d->decim < 0 || d->decim > ehi::kMaxDecim) return bad("decim must be in [0, 64]");
  if (d->decim >= 2) {
    if (d->weighting != EHI_WEIGHT_FINITE_RECORD)
      return bad("time-axis resampling applies to the finite-record weighting");
    if (d->windows == 2) return bad("time-axis resampling needs one staging window");
    const int K = decim_half_length(d->decim, d->dt, max_freq(d));
    if (K < 0) return bad("decimation factor too large for the highest frequency (1/(D dt) must exceed 2 f_max)");
    if (K > ehi::kMaxDecimK) return bad("resampling filter longer than 1025 taps");
    const int chunk = d->chunk ? d->chunk : 256;
    if (2 * K > chunk || 2 * d->decim > chunk)
      return bad("staging window shorter than the resampling filter (raise chunk)");
  }
  const long long chunk = d->chunk ? d->chunk : 256;
  if ((nsub + 256) * chunk * 4 >= (1LL << 31)) return bad("subgrid too large for the staging buffer");
  return true;
}

ehi::Geometry make_geometry(const ehi_survey_desc* d) {
  ehi::Geometry g{};
  g.nz = d->nz;
  g.nx = d->nx;
  g.nb = d->nb;
  g.Z = d->nz + 2 * d->nb;
  g.X = d->nx + 2 * d->nb;
  g.Zp = g.Z + 2 * ehi::kGhost;
  g.Xp = (int)ehi::align_up((size_t)g.X + 2 * ehi::kGhost, ehi::kRowAlign);
  g.stride = d->stride;
  g.sshift = d->stride == 1 ? 0 : d->stride == 2 ? 1 : d->stride == 4 ? 2 : 3;
  g.nzs = ehi::cdiv(d->nz, d->stride);
  g.nxs = ehi::cdiv(d->nx, d->stride);
  g.nsub = g.nzs * g.nxs;
  g.nsub_p = (int)ehi::align_up((size_t)g.nsub, 256);  // the DFT reads whole 256-point blocks
  g.chunk = d->chunk ? d->chunk : 256;
  g.windows = d->windows == 2 ? 2 : 1;
  g.nt = d->nt;
  g.nr = d->nr;
  g.nf = d->nf;
  g.nrb = d->nr_batch > 0 ? std::min(d->nr_batch, d->nr) : d->nr;
  g.max_ns = d->max_ns;
  g.h = d->h;
  g.dt = d->dt;
  g.split_bf16 = d->precision == EHI_PREC_SPLIT_BF16 ? 1 : 0;
  g.weighting = d->weighting;
  g.keep_z = d->keep_z;
  g.keep_x = d->keep_x;
  // compressed surveys hold one receiver batch's spectra at a time: each batch
  // is transformed into the compressed spectra as soon as its DFT is complete
  g.gh_rows = g.keep_z > 0 ? g.nrb : g.nr;
  // the three-part BF16 DFT: FP32-equivalent operands, faster than the FP32
  // matrix-core form and with half its element-wise error (measured)
  g.dft_form = 1;
  if (const char* e = std::getenv("EHI_DFT_FORM")) {
    int v = std::atoi(e);
    if (v == 0 || v == 1) g.dft_form = v;
  }
  g.decim = 1;
  g.dK = 0;
  g.dM = d->nt;
  g.dqa = 0;
  g.dqb = d->nt - 1;
  g.dhist = 0;
  g.drows = 0;
  if (d->decim >= 2) {
    // kept samples n_q = 1 - K + q D whose filter support [n_q - K, n_q + K]
    // meets the record 1..nt
    g.decim = d->decim;
    g.dK = decim_half_length(d->decim, d->dt, max_freq(d));
    g.dM = (d->nt - 1 + 2 * g.dK) / g.decim + 1;
    g.dqa = ehi::cdiv(g.dK, g.decim);                   // first q with n_q >= 1
    g.dqb = (d->nt - 1 + g.dK) / g.decim;               // last q with n_q <= nt
    g.dhist = 2 * g.dK;
    const int chunk = d->chunk ? d->chunk : 256;
    g.drows = chunk / g.decim + ehi::cdiv(2 * g.dK, g.decim) + 2;
  }
  g.herk_form = d->herk_form;
  // 64 x 64 tile pairs, except the plain form's vector-unit kernel (32 x 32)
  int ntile = ehi::cdiv(g.nr, (!g.split_bf16 && g.herk_form == 3) ? ehi::kHerkTile : 64);
  int pairs = ntile * (ntile + 1) / 2;
  int want = ehi::cdiv(2048, pairs * g.nf);
  // the final-spectrum split-BF16 contraction runs one workgroup per CU per
  // (frequency, partition, pair group or tile): partitions for about four full
  // rounds of workgroups (a partial last round costs a round)
  g.herk_whole = (g.split_bf16 && g.weighting == EHI_WEIGHT_LONG_RECORD) ? 1 : 0;
  if (g.herk_whole) want = std::max(1, 1024 / (g.nf * ehi::herk_whole_groups(g.nr)));
  if (d->herk_form == 2) g.herk_whole = 0;
  if (g.herk_whole == 0 && d->herk_form == 2) want = ehi::cdiv(2048, pairs * g.nf);
  int kmax = std::max(1, g.nsub / 1024);
  g.herk_split = std::max(1, std::min(want, std::min(ehi::kHerkSplitMax, kmax)));
  // accuracy floor (at most kHerkMaxStages stages per partition): at 75,000
  // grid points it takes 59 partitions and cuts the multipliers' error at
  // 3 Hz from 6.5e-6 to 2.1e-6 against the FP64 oracle for 4 % more time in
  // the contraction
  const int stage_floor = std::min(ehi::kHerkSplitMax, ehi::cdiv(ehi::cdiv(g.nsub, 32), ehi::kHerkMaxStages));
  g.herk_split = std::max(g.herk_split, stage_floor);
  if (d->herk_split > 0) g.herk_split = d->herk_split;
  g.tblock = 8;
  g.seg_rows = 256;  // measured best for the 1000 x 300 benchmark grid (1-2 % over 128)
  // tuning overrides (launch shapes only; results do not depend on them)
  if (const char* e = std::getenv("EHI_TBLOCK")) {
    int v = std::atoi(e);
    if (v == 4 || v == 8) g.tblock = v;
  }
  if (const char* e = std::getenv("EHI_HERK_WHOLE")) {
    if (std::atoi(e) == 0 && g.herk_whole) {
      g.herk_whole = 0;
      g.herk_split = std::max(1, std::min(ehi::cdiv(2048, pairs * g.nf), std::min(ehi::kHerkSplitMax, kmax)));
      g.herk_split = std::max(g.herk_split, stage_floor);
    }
  }
  if (const char* e = std::getenv("EHI_HERK_SPLIT")) {
    int v = std::atoi(e);
    if (v >= 1 && v <= ehi::kHerkSplitMax) g.herk_split = v;
  }
  if (const char* e = std::getenv("EHI_SEG_ROWS")) {
    int v = std::atoi(e);
    if (v >= ehi::kMinSegRows && v <= ehi::kMaxSegRows) g.seg_rows = v;
  }
  g.band_req = 0;
  if (const char* e = std::getenv("EHI_BAND")) {
    int v = std::atoi(e);
    if (v == 256 || v == 384 || v == 448 || v == 512) g.band_req = v;
  }
  g.band = g.band_req ? g.band_req : ehi::march_band_for(g.X, g.tblock);
  return g;
}

ehi::Layout make_layout(const ehi::Geometry& g) {
  ehi::Layout L{};
  size_t off = 0;
  auto take = [&](size_t bytes) {
    size_t o = off;
    off = ehi::align_up(off + bytes, ehi::kAlign);
    return o;
  };
  const size_t nn = (size_t)g.nr * g.nr;
  L.freq = take(sizeof(double) * g.nf);
  L.rec = take(sizeof(int32_t) * 2 * g.nr);
  L.ca = take(sizeof(float) * g.plane());
  L.bd = take(sizeof(float) * (ehi::kMaxSponge + 1));
  L.rowtab = take(sizeof(ehi::RowEntry) * (size_t)ehi::cdiv(g.Z, ehi::kMinSegRows) * ehi::kRowTabStride);
  L.rowrec = take(sizeof(int32_t) * (size_t)g.Z);
  L.recmap = take(sizeof(int32_t) * g.plane());
  L.vmax = take(sizeof(uint32_t) * 4);
  L.tw = take(sizeof(float2) * (size_t)g.nt * g.nf);
  L.u0 = take(sizeof(float) * g.plane() * g.nrb);
  L.u1 = take(sizeof(float) * g.plane() * g.nrb);
  L.w0 = take(sizeof(float) * g.plane() * g.nrb);
  L.w1 = take(sizeof(float) * g.plane() * g.nrb);
  L.stage = take(sizeof(float) * (size_t)g.windows * g.nrb * g.chunk * g.nsub_p);
  L.ghat = take(sizeof(float2) * (size_t)g.nf * g.gh_rows * g.nsub);
  L.hpart = take(sizeof(float2) * (size_t)g.herk_split * g.nf * nn);
  L.hpart64 = take(g.weighting == EHI_WEIGHT_FINITE_RECORD ? sizeof(double2) * (size_t)g.herk_split * g.nf * nn : 0);
  L.r2scale = take(sizeof(double) * g.nf);
  L.gscale = take(sizeof(double) * g.nf);
  const bool dec = g.decim > 1;
  L.dtaps = take(dec ? sizeof(float) * (2 * g.dK + 1) : 0);
  L.dtw = take(dec ? sizeof(float2) * (size_t)g.dM * g.nf : 0);
  L.dhistbuf = take(dec ? sizeof(float) * (size_t)g.nrb * g.dhist * g.nsub_p : 0);
  L.ddec = take(dec ? sizeof(float) * (size_t)g.nrb * g.drows * g.nsub_p : 0);
  L.dctz = take(sizeof(float2) * (size_t)g.keep_z * g.nzs);
  L.dctx = take(sizeof(float2) * (size_t)g.keep_x * g.nxs);
  L.dtmp = take(sizeof(float2) * (size_t)g.nf * g.gh_rows * g.nxs * g.keep_z);
  L.gcomp = take(sizeof(float2) * (size_t)g.nf * g.nr * g.keep_z * g.keep_x);
  L.hhat = take(sizeof(double2) * g.nf * nn);
  L.qhat = take(sizeof(double2) * g.nf * nn);
  L.lfac = take(sizeof(double2) * g.nf * nn);
  L.lfac32 = take(sizeof(float2) * g.nf * nn);
  const size_t np = (size_t)ehi::solve_blocks(g) * 32;
  L.m64 = take(sizeof(double2) * (size_t)g.nf * np * np);
  L.m32 = take(sizeof(float2) * (size_t)g.nf * np * np);
  L.y32 = take(sizeof(float2) * (size_t)g.nf * g.max_ns * g.nr);
  L.r32 = take(sizeof(float2) * (size_t)g.nf * g.max_ns * g.nr);
  L.x64 = take(sizeof(double2) * (size_t)g.nf * g.max_ns * g.nr);
  L.status = take(sizeof(int32_t) * (g.nf + 4));
  L.eig = take(sizeof(double) * g.nf);
  L.jobs = take(sizeof(ehi::FactorJob) * g.nf);
  L.total = off;
  return L;
}

}  // namespace

namespace ehi {

hipError_t Profiler::begin(int kind, hipStream_t st) {
  if (!on) return hipSuccess;
  if (open_kind == kind && open_stream == st) return hipSuccess;
  hipError_t e = end();
  if (e != hipSuccess) return e;
  if ((e = hipEventCreate(&open_start)) != hipSuccess) return e;
  if ((e = hipEventRecord(open_start, st)) != hipSuccess) return e;
  open_kind = kind;
  open_stream = st;
  open_launches = 0;
  return hipSuccess;
}

hipError_t Profiler::end() {
  if (open_kind < 0) return hipSuccess;
  hipEvent_t stop;
  hipError_t e = hipEventCreate(&stop);
  if (e == hipSuccess) e = hipEventRecord(stop, open_stream);
  if (e == hipSuccess) recs.push_back(ProfRecord{open_kind, open_launches, open_start, stop});
  open_kind = -1;
  open_launches = 0;
  open_start = nullptr;
  return e;
}

}  // namespace ehi

namespace {

// The second stream and its events (two staging windows); safe on a partly
// created survey.
void release_side(ehi_survey* s) {
  for (int b = 0; b < 2; ++b) {
    if (s->ev_marched[b]) (void)hipEventDestroy(s->ev_marched[b]);
    if (s->ev_dft[b]) (void)hipEventDestroy(s->ev_dft[b]);
    s->ev_marched[b] = s->ev_dft[b] = nullptr;
  }
  if (s->side) (void)hipStreamDestroy(s->side);
  s->side = nullptr;
}

}  // namespace

#define PROF(kind, st) EHI_TRY(s->prof.begin((kind), (st)), "profiler event")
#define PROF_N(n) s->prof.count(n)
#define PROF_END() EHI_TRY(s->prof.end(), "profiler event")

extern "C" {

const char* ehi_last_error(void) { return g_err.c_str(); }

const char* ehi_version(void) { return "ehi 0.1 gfx950"; }

size_t ehi_workspace_bytes(const ehi_survey_desc* desc) {
  std::string why;
  if (!validate(desc, &why)) {
    g_err = why;
    return 0;
  }
  return make_layout(make_geometry(desc)).total;
}

ehi_status ehi_create(const ehi_survey_desc* desc, void* workspace_dev, size_t ws_bytes,
                      void* stream, ehi_survey** out) {
  g_err.clear();
  if (!out) return fail(EHI_EINVAL, "out is NULL");
  *out = nullptr;
  std::string why;
  if (!validate(desc, &why)) return fail(EHI_EINVAL, why);
  if (!workspace_dev) return fail(EHI_EINVAL, "workspace is NULL");
  if (reinterpret_cast<uintptr_t>(workspace_dev) % ehi::kAlign != 0)
    return fail(EHI_EINVAL, "workspace must be 256-byte aligned");
  ehi::Geometry g = make_geometry(desc);
  ehi::Layout L = make_layout(g);
  if (ws_bytes < L.total)
    return fail(EHI_ENOMEM, "workspace has " + std::to_string(ws_bytes) + " bytes, needs " +
                                std::to_string(L.total));
  ehi_survey* s = new (std::nothrow) ehi_survey();
  if (!s) return fail(EHI_ENOMEM, "host allocation failed");
  s->g = g;
  s->L = L;
  s->precision = desc->precision;
  s->rec_iz.assign(desc->rec_iz, desc->rec_iz + desc->nr);
  s->rec_ix.assign(desc->rec_ix, desc->rec_ix + desc->nr);
  s->freq.assign(desc->freq_hz, desc->freq_hz + desc->nf);
  s->ws = static_cast<char*>(workspace_dev);
  s->ws_bytes = ws_bytes;
  s->stream = static_cast<hipStream_t>(stream);
  s->state = ehi::State::Created;
  s->medium = false;
  s->mu = 0.0;
  // one FP64-residual refinement step in the split-BF16 form: after it the
  // error is about (cond * 2^-24)^2 of the solution, far below the complex64
  // output's rounding at the conditioning of the penalised Hessians (a second
  // step changed no printed digit of the full-size error against the oracle)
  s->refine = desc->precision == EHI_PREC_SPLIT_BF16 ? 1 : 0;
  hipError_t e = hipGetDevice(&s->device);
  if (e != hipSuccess) {
    delete s;
    return hip_fail(e, "hipGetDevice");
  }
  std::vector<int32_t> rec(2 * g.nr);
  std::copy(s->rec_iz.begin(), s->rec_iz.end(), rec.begin());
  std::copy(s->rec_ix.begin(), s->rec_ix.end(), rec.begin() + g.nr);
  e = hipMemcpyAsync(s->ptr<double>(L.freq), s->freq.data(), sizeof(double) * g.nf,
                     hipMemcpyHostToDevice, s->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(s->ptr<int32_t>(L.rec), rec.data(), sizeof(int32_t) * 2 * g.nr,
                       hipMemcpyHostToDevice, s->stream);
  // receiver map of the padded plane (index, -1 elsewhere) and the rows holding
  // receivers, for the modelling runs on the marching kernel
  std::vector<int32_t> recmap(g.plane(), -1), rowrec(g.Z, 0);
  s->rec_distinct = true;
  for (int r = 0; r < g.nr; ++r) {
    const int q = s->rec_iz[r] + g.nb;
    const size_t o = (size_t)(q + ehi::kGhost) * g.Xp + (s->rec_ix[r] + g.nb + ehi::kGhost);
    if (recmap[o] >= 0) s->rec_distinct = false;
    recmap[o] = r;
    rowrec[q] = 1;
  }
  if (e == hipSuccess)
    e = hipMemcpyAsync(s->ptr<int32_t>(L.recmap), recmap.data(), sizeof(int32_t) * recmap.size(),
                       hipMemcpyHostToDevice, s->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(s->ptr<int32_t>(L.rowrec), rowrec.data(), sizeof(int32_t) * rowrec.size(),
                       hipMemcpyHostToDevice, s->stream);
  if (e == hipSuccess) e = ehi::launch_twiddles(g, s->ptr<double>(L.freq), s->ptr<float2>(L.tw), s->stream);
  // finite-record Gram scale per frequency; with time-axis resampling the
  // filter taps, the twiddles at the kept samples and D / H(w)
  std::vector<double> r2scale(g.nf, 1.0 / g.nt), gscale(g.nf, 1.0);
  std::vector<float> taps32;
  if (g.decim > 1) {
    const std::vector<double> h = decim_taps(g.decim, g.dK);
    taps32.assign(h.begin(), h.end());
    for (int f = 0; f < g.nf; ++f) {
      const double w = 2.0 * 3.14159265358979323846 * s->freq[f];
      double H = h[g.dK];
      for (int j = 1; j <= g.dK; ++j) H += 2.0 * h[g.dK + j] * std::cos(w * j * g.dt);
      gscale[f] = g.decim / H;
      r2scale[f] = gscale[f] * gscale[f] * g.decim / g.nt;
    }
    if (e == hipSuccess)
      e = hipMemcpyAsync(s->ptr<float>(L.dtaps), taps32.data(), sizeof(float) * taps32.size(),
                         hipMemcpyHostToDevice, s->stream);
    if (e == hipSuccess)
      e = ehi::launch_twiddles_at(g.dM, g.nf, g.dt, s->ptr<double>(L.freq), 1 - g.dK, g.decim,
                                  s->ptr<float2>(L.dtw), s->stream);
  }
  if (e == hipSuccess)
    e = hipMemcpyAsync(s->ptr<double>(L.r2scale), r2scale.data(), sizeof(double) * g.nf, hipMemcpyHostToDevice,
                       s->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(s->ptr<double>(L.gscale), gscale.data(), sizeof(double) * g.nf, hipMemcpyHostToDevice,
                       s->stream);
  if (e == hipSuccess && g.keep_z > 0) {
    e = ehi::launch_dct_matrix(g.nzs, g.keep_z, s->ptr<float2>(L.dctz), s->stream);
    if (e == hipSuccess) e = ehi::launch_dct_matrix(g.nxs, g.keep_x, s->ptr<float2>(L.dctx), s->stream);
  }
  if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
  if (e == hipSuccess && g.windows == 2) {
    e = hipStreamCreateWithFlags(&s->side, hipStreamNonBlocking);
    for (int b = 0; b < 2 && e == hipSuccess; ++b) {
      e = hipEventCreateWithFlags(&s->ev_marched[b], hipEventDisableTiming);
      if (e == hipSuccess) e = hipEventCreateWithFlags(&s->ev_dft[b], hipEventDisableTiming);
    }
  }
  if (e != hipSuccess) {
    release_side(s);
    delete s;
    return hip_fail(e, "ehi_create set-up");
  }
  *out = s;
  return EHI_OK;
}

ehi_status ehi_destroy(ehi_survey* s) {
  if (!s) return EHI_OK;
  (void)s->prof.end();
  for (auto& r : s->prof.recs) {
    (void)hipEventDestroy(r.start);
    (void)hipEventDestroy(r.stop);
  }
  release_side(s);
  delete s;
  return EHI_OK;
}

ehi_status ehi_profile_enable(ehi_survey* s, int enable) {
  g_err.clear();
  if (!s) return fail(EHI_EINVAL, "survey is NULL");
  if (!enable) PROF_END();
  s->prof.on = enable != 0;
  return EHI_OK;
}

ehi_status ehi_profile_read(ehi_survey* s, double* ms, int64_t* launches) {
  g_err.clear();
  if (!s || !ms || !launches) return fail(EHI_EINVAL, "NULL argument");
  PROF_END();
  for (int k = 0; k < EHI_PROF_KINDS; ++k) {
    ms[k] = 0.0;
    launches[k] = 0;
  }
  hipError_t first = hipSuccess;
  for (auto& r : s->prof.recs) {
    hipError_t e = hipEventSynchronize(r.stop);
    float t = 0.f;
    if (e == hipSuccess) e = hipEventElapsedTime(&t, r.start, r.stop);
    if (e != hipSuccess && first == hipSuccess) first = e;
    if (r.kind >= 0 && r.kind < EHI_PROF_KINDS) {
      ms[r.kind] += t;
      launches[r.kind] += r.launches;
    }
    (void)hipEventDestroy(r.start);
    (void)hipEventDestroy(r.stop);
  }
  s->prof.recs.clear();
  if (first != hipSuccess) return hip_fail(first, "profile read");
  return EHI_OK;
}

ehi_status ehi_build_green(ehi_survey* s, const float* vel_dev) {
  g_err.clear();
  if (!s) return fail(EHI_EINVAL, "survey is NULL");
  if (!vel_dev) return fail(EHI_EINVAL, "velocity is NULL");
  const ehi::Geometry& g = s->g;
  const ehi::Layout& L = s->L;
  hipStream_t st = s->stream;
  uint32_t* vmax = s->ptr<uint32_t>(L.vmax);
  float* ca = s->ptr<float>(L.ca);
  float* bd = s->ptr<float>(L.bd);
  PROF(EHI_PROF_SETUP, st);
  EHI_TRY(ehi::launch_vmax(vel_dev, g.nz * g.nx, vmax, st), "vmax");
  EHI_TRY(ehi::launch_coefficients(g, vel_dev, vmax, ca, bd, st), "coefficients");
  s->medium = true;
  ehi::RowEntry* rowtab = s->ptr<ehi::RowEntry>(L.rowtab);
  EHI_TRY(ehi::launch_row_table(g, bd, s->ptr<int32_t>(L.rowrec), rowtab, st), "row table");
  PROF_N(4);
  const float2* tw = s->ptr<float2>(L.tw);
  float2* ghat = s->ptr<float2>(L.ghat);
  const size_t wfloats = (size_t)g.nrb * g.chunk * g.nsub_p;
  float* stage[2] = {s->ptr<float>(L.stage), s->ptr<float>(L.stage) + (g.windows == 2 ? wfloats : 0)};
  // with two windows the DFT of window buffer b runs on the side stream once
  // the steps filling it are done (ev_marched[b]); steps into b wait until
  // that DFT has read it (ev_dft[b])
  const bool two = g.windows == 2;
  hipStream_t dst = two ? s->side : st;
  bool pending[2] = {false, false};
  // the finite-record contraction reads whole 32-point blocks of staged samples;
  // the tail of the last block lies in the row padding, which must hold zeros
  if (g.weighting == EHI_WEIGHT_FINITE_RECORD)
    EHI_TRY(ehi::launch_zero_stage_tails(g, s->ptr<float>(L.stage), st), "staging padding");
  auto free_window = [&](int b) -> hipError_t {
    if (!two || !pending[b]) return hipSuccess;
    pending[b] = false;
    return hipStreamWaitEvent(st, s->ev_dft[b], 0);
  };
  const bool resample = g.weighting == EHI_WEIGHT_FINITE_RECORD && g.decim > 1;
  // the kept-sample buffer as a staging buffer of drows rows per receiver
  ehi::Geometry gd = g;
  gd.chunk = g.drows;
  // the spectra buffer as the DFT sees it (one batch's rows when compressed)
  ehi::Geometry gb = g;
  gb.nr = g.gh_rows;
  const float2* dtw = s->ptr<float2>(L.dtw);
  float* ddec = s->ptr<float>(L.ddec);
  for (int r0 = 0; r0 < g.nr; r0 += g.nrb) {
    const int nb_now = std::min(g.nrb, g.nr - r0);
    int q_done = 0;  // kept samples already produced (resampling)
    float* ub[2] = {s->ptr<float>(L.u0), s->ptr<float>(L.u1)};
    float* wb[2] = {s->ptr<float>(L.w0), s->ptr<float>(L.w1)};
    int b = 0;  // window buffer being filled
    EHI_TRY(free_window(0), "window wait");
    PROF(EHI_PROF_SETUP, st);
    EHI_TRY(ehi::launch_wave_init(g, vel_dev, s->ptr<int32_t>(L.rec), r0, nb_now, ub[0], wb[0],
                                  stage[0], st),
            "wave init");
    // the marching kernel relies on zero ghost rings in both ping-pong buffers
    const size_t nplane = (size_t)nb_now * g.plane();
    EHI_TRY(ehi::launch_fill_u32(reinterpret_cast<uint32_t*>(ub[1]), 0u, nplane, st), "fill");
    EHI_TRY(ehi::launch_fill_u32(reinterpret_cast<uint32_t*>(wb[1]), 0u, nplane, st), "fill");
    PROF_N(4);
    // sample n_cur sits in (ub[cur], wb[cur]) and in staging slot (n_cur - 1) % chunk
    int cur = 0;
    int n_cur = 1;
    for (;;) {
      if (n_cur % g.chunk == 0 || n_cur == g.nt) {
        const int n0 = (n_cur - 1) / g.chunk * g.chunk + 1;
        if (two) {
          EHI_TRY(hipEventRecord(s->ev_marched[b], st), "window event");
          EHI_TRY(hipStreamWaitEvent(dst, s->ev_marched[b], 0), "window wait");
        }
        if (resample) {
          // kept samples whose filter support ends in this window (all that
          // remain at the end of the record), then the running spectra and
          // their Gram on them; the window's last 2K samples are kept for the
          // next window's filter
          const bool last = n_cur == g.nt;
          const int q_hi = last ? g.dM : std::min(g.dM, (n_cur - 1) / g.decim + 1);
          const int cnt = q_hi - q_done;
          if (cnt > 0) {
            PROF(EHI_PROF_DFT, dst);
            EHI_TRY(ehi::launch_decimate(g, stage[b], s->ptr<float>(L.dhistbuf), s->ptr<float>(L.dtaps), q_done, cnt,
                                         n0, n_cur, nb_now, ddec, dst),
                    "resampling filter");
            PROF_N(1);
            PROF(EHI_PROF_HERK, dst);
            EHI_TRY(ehi::launch_herk_r2_chunk(gd, ddec, dtw, ghat, q_done + 1, cnt, q_done == 0, g.dqa - q_done,
                                              g.dqb - q_done, s->ptr<double2>(L.hpart64), dst),
                    "finite-record contraction");
            PROF_N(1);
            PROF(EHI_PROF_DFT, dst);
            EHI_TRY(ehi::launch_dft_chunk(gd, ddec, dtw, q_done + 1, cnt, q_done == 0, r0, nb_now, ghat, dst),
                    "dft chunk");
            PROF_N(1);
            q_done = q_hi;
          }
          if (!last)
            EHI_TRY(ehi::launch_hist_copy(g, stage[b], n_cur, nb_now, s->ptr<float>(L.dhistbuf), dst),
                    "resampling history");
        } else {
          if (g.weighting == EHI_WEIGHT_FINITE_RECORD) {
            // the running spectra of this window, before the DFT advances them
            PROF(EHI_PROF_HERK, dst);
            EHI_TRY(ehi::launch_herk_r2_chunk(g, stage[b], tw, ghat, n0, n_cur - n0 + 1, n0 == 1, 0,
                                              n_cur - n0, s->ptr<double2>(L.hpart64), dst),
                    "finite-record contraction");
            PROF_N(1);
          }
          PROF(EHI_PROF_DFT, dst);
          if (g.keep_z > 0) {
            // the batch's own rows of the spectra buffer
            EHI_TRY(ehi::launch_dft_chunk(gb, stage[b], tw, n0, n_cur - n0 + 1, n0 == 1, 0, nb_now, ghat, dst),
                    "dft chunk");
          } else {
            EHI_TRY(ehi::launch_dft_chunk(g, stage[b], tw, n0, n_cur - n0 + 1, n0 == 1, r0, nb_now, ghat, dst),
                    "dft chunk");
          }
          PROF_N(1);
          if (g.keep_z > 0 && n_cur == g.nt) {
            // the batch's spectra are complete: into the compressed spectra
            PROF(EHI_PROF_HERK, dst);
            EHI_TRY(ehi::launch_dct_compress(g, ghat, g.gh_rows, r0, nb_now, s->ptr<float2>(L.dctz),
                                             s->ptr<float2>(L.dctx), s->ptr<float2>(L.dtmp),
                                             s->ptr<float2>(L.gcomp), dst),
                    "spatial compression");
            PROF_N(2 * g.nf);
          }
        }
        if (two) {
          EHI_TRY(hipEventRecord(s->ev_dft[b], dst), "window event");
          pending[b] = true;
          b ^= 1;
          if (n_cur != g.nt) EHI_TRY(free_window(b), "window wait");
        }
      }
      if (n_cur == g.nt) break;
      // advance to the next multiple of tblock (never past the chunk end: tblock | chunk)
      const int target = std::min(g.nt, (n_cur / g.tblock + 1) * g.tblock);
      PROF(EHI_PROF_STEP, st);
      EHI_TRY(ehi::launch_march(g, ca, bd, rowtab, ub[cur], wb[cur], ub[1 - cur], wb[1 - cur], stage[b],
                                n_cur % g.chunk, target - n_cur, nb_now, st),
              "time steps");
      PROF_N(1);
      cur = 1 - cur;
      n_cur = target;
    }
  }
  // the survey's stream resumes after the last DFT
  EHI_TRY(free_window(0), "window wait");
  EHI_TRY(free_window(1), "window wait");
  if (resample) {
    // the resampled running spectra to the record's spectra: times D / H(w)
    PROF(EHI_PROF_DFT, st);
    EHI_TRY(ehi::launch_scale_spectra(g, s->ptr<double>(L.gscale), ghat, st), "spectra scale");
    PROF_N(1);
  }
  PROF_END();
  s->state = ehi::State::Green;
  return EHI_OK;
}

ehi_status ehi_build_hessian(ehi_survey* s) {
  g_err.clear();
  if (!s) return fail(EHI_EINVAL, "survey is NULL");
  if (s->state < ehi::State::Green) return fail(EHI_ESTATE, "build_hessian before build_green");
  const ehi::Geometry& g = s->g;
  const ehi::Layout& L = s->L;
  float2* hpart = s->ptr<float2>(L.hpart);
  PROF(EHI_PROF_HERK, s->stream);
  if (g.weighting == EHI_WEIGHT_FINITE_RECORD) {
    // accumulated during build_green; only the reduction remains
    EHI_TRY(ehi::launch_herk_r2_reduce(g, s->ptr<double2>(L.hpart64), s->ptr<double>(L.r2scale),
                                       s->ptr<double2>(L.hhat), s->stream),
            "finite-record reduce");
    PROF_N(1);
    PROF_END();
    s->state = ehi::State::Hessian;
    return EHI_OK;
  }
  const float2* spectra = s->ptr<float2>(L.ghat);
  if (g.keep_z > 0) {
    // over the leading 2D DCT-II coefficients of each spectrum row; they hold
    // the energy in few terms, where the split-BF16 form's per-term rounding no
    // longer averages out, so this contraction sums FP32 products in FP64
    // (either precision mode)
    // (the compressed spectra were formed batch by batch in build_green or
    // load_green_dft)
    EHI_TRY(ehi::launch_herk_compressed(g, s->ptr<float2>(L.gcomp), g.keep_z * g.keep_x,
                                        s->ptr<double2>(L.hhat), s->stream),
            "compressed contraction");
    PROF_N(2);
    PROF_END();
    s->state = ehi::State::Hessian;
    return EHI_OK;
  }
  // over the subgrid points
  if (s->precision == EHI_PREC_SPLIT_BF16) {
    EHI_TRY(ehi::launch_herk_split_bf16(g, spectra, hpart, s->stream), "herk bf16");
  } else {
    EHI_TRY(ehi::launch_herk_fp32(g, spectra, hpart, s->stream), "herk fp32");
  }
  EHI_TRY(ehi::launch_herk_reduce(g, hpart, s->ptr<double2>(L.hhat), s->stream), "herk reduce");
  PROF_N(2);
  PROF_END();
  s->state = ehi::State::Hessian;
  return EHI_OK;
}

ehi_status ehi_factor(ehi_survey* s, double mu, int32_t* bad_freq) {
  ehi_survey* one[1] = {s};
  void* ws = s ? s->ws + s->L.jobs : nullptr;
  const size_t bytes = s ? sizeof(ehi::FactorJob) * s->g.nf : 0;
  int32_t bad_s = -1;
  return ehi_factor_batch(one, 1, &mu, ws, bytes, s ? s->stream : nullptr, &bad_s, bad_freq);
}

size_t ehi_batch_workspace_bytes(ehi_survey* const* surveys, int32_t n) {
  if (!surveys || n < 1) {
    g_err = "no surveys";
    return 0;
  }
  size_t jobs = 0;
  for (int k = 0; k < n; ++k) {
    if (!surveys[k]) {
      g_err = "NULL survey in the batch";
      return 0;
    }
    jobs += surveys[k]->g.nf;
  }
  return ehi::align_up(sizeof(ehi::FactorJob) * jobs, ehi::kAlign);
}

}  // extern "C"

namespace {

// The batched factorisation with its job table at djobs_raw (capacity
// cap_bytes, device memory of the current device).
ehi_status factor_batch_impl(ehi_survey* const* surveys, int32_t n, const double* mu, void* djobs_raw,
                             size_t cap_bytes, void* stream, int32_t* bad_survey, int32_t* bad_freq) {
  g_err.clear();
  if (bad_survey) *bad_survey = -1;
  if (bad_freq) *bad_freq = -1;
  if (!surveys || n < 1 || !mu) return fail(EHI_EINVAL, "no surveys or no mu");
  std::vector<ehi::FactorJob> jobs;
  int max_nr = 0;
  for (int k = 0; k < n; ++k) {
    ehi_survey* s = surveys[k];
    if (!s) return fail(EHI_EINVAL, "survey is NULL");
    if (s->state < ehi::State::Hessian) return fail(EHI_ESTATE, "factor before build_hessian");
    if (!(mu[k] > 0) || !std::isfinite(mu[k])) return fail(EHI_EINVAL, "mu must be positive and finite");
    const ehi::Geometry& g = s->g;
    const ehi::Layout& L = s->L;
    const size_t nn = (size_t)g.nr * g.nr;
    const size_t npp = (size_t)ehi::solve_blocks(g) * 32 * ehi::solve_blocks(g) * 32;
    for (int f = 0; f < g.nf; ++f) {
      ehi::FactorJob j;
      j.hhat = s->ptr<double2>(L.hhat) + f * nn;
      j.qhat = s->ptr<double2>(L.qhat) + f * nn;
      j.lfac = s->ptr<double2>(L.lfac) + f * nn;
      j.l32 = s->ptr<float2>(L.lfac32) + f * nn;
      j.m64 = s->ptr<double2>(L.m64) + f * npp;
      j.m32 = s->ptr<float2>(L.m32) + f * npp;
      j.status = s->ptr<int32_t>(L.status) + f;
      j.mu = mu[k];
      j.nr = g.nr;
      j.fp64 = s->precision == EHI_PREC_SPLIT_BF16 ? 1 : 0;
      jobs.push_back(j);
    }
    max_nr = std::max(max_nr, g.nr);
  }
  if (!djobs_raw || cap_bytes < sizeof(ehi::FactorJob) * jobs.size())
    return fail(EHI_ENOMEM, "batch workspace too small");
  hipStream_t st = static_cast<hipStream_t>(stream);
  ehi_survey* s = surveys[0];
  ehi::FactorJob* djobs = static_cast<ehi::FactorJob*>(djobs_raw);
  PROF(EHI_PROF_FACTOR, st);
  EHI_TRY(hipMemcpyAsync(djobs, jobs.data(), sizeof(ehi::FactorJob) * jobs.size(),
                         hipMemcpyHostToDevice, st),
          "job table upload");
  EHI_TRY(ehi::launch_factor_jobs(djobs, (int)jobs.size(), st), "factor");
  EHI_TRY(ehi::launch_minv_jobs(djobs, (int)jobs.size(), max_nr, st), "triangular inverses");
  PROF_N(3);
  PROF_END();
  // status readback (the only wait): one small copy per survey
  std::vector<std::vector<int32_t>> host(n);
  for (int k = 0; k < n; ++k) {
    host[k].assign(surveys[k]->g.nf, 0);
    EHI_TRY(hipMemcpyAsync(host[k].data(), surveys[k]->ptr<int32_t>(surveys[k]->L.status),
                           sizeof(int32_t) * surveys[k]->g.nf, hipMemcpyDeviceToHost, st),
            "status readback");
  }
  EHI_TRY(hipStreamSynchronize(st), "factor sync");
  ehi_status result = EHI_OK;
  for (int k = 0; k < n; ++k) {
    surveys[k]->state = ehi::State::Hessian;
    bool ok = true;
    for (int f = 0; f < surveys[k]->g.nf; ++f) {
      if (host[k][f] != 0) {
        if (result == EHI_OK) {
          if (bad_survey) *bad_survey = k;
          if (bad_freq) *bad_freq = f;
          result = fail(EHI_ENOTPD, "Qhat not positive definite: survey " + std::to_string(k) +
                                        ", frequency index " + std::to_string(f));
        }
        ok = false;
        break;
      }
    }
    if (ok) {
      surveys[k]->mu = mu[k];
      surveys[k]->state = ehi::State::Factored;
    }
  }
  return result;
}

// Job table of the batched factorisation for callers that cannot allocate:
// one copy per device, held until the process ends.  Host code never passes
// the array's name to a kernel or a copy: each device's address comes from
// hipGetSymbolAddress, taken once per device with that device current.
constexpr size_t kStaticJobs = 4096;
static __device__ __align__(256) unsigned char scratch[kStaticJobs * sizeof(ehi::FactorJob)];
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

ehi_status scratch_for_current_device(void** out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  if (dev < 0 || dev >= kMaxDevices) return fail(EHI_EINVAL, "device index beyond the static table");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
    if (!p) return fail(EHI_EHIP, "hipGetSymbolAddress returned NULL");
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return EHI_OK;
}

}  // namespace

extern "C" {

ehi_status ehi_factor_batch(ehi_survey* const* surveys, int32_t n, const double* mu, void* batch_ws,
                            size_t ws_bytes, void* stream, int32_t* bad_survey, int32_t* bad_freq) {
  return factor_batch_impl(surveys, n, mu, batch_ws, ws_bytes, stream, bad_survey, bad_freq);
}

ehi_status ehi_factor_batch_static(ehi_survey* const* surveys, int32_t n, const double* mu, void* stream,
                                   int32_t* bad_survey, int32_t* bad_freq) {
  g_err.clear();
  if (bad_survey) *bad_survey = -1;
  if (bad_freq) *bad_freq = -1;
  if (!surveys || n < 1 || !mu) return fail(EHI_EINVAL, "no surveys or no mu");
  size_t jobs = 0;
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  for (int k = 0; k < n; ++k) {
    if (!surveys[k]) return fail(EHI_EINVAL, "survey is NULL");
    if (surveys[k]->device != dev) return fail(EHI_EINVAL, "every survey must live on the current device");
    jobs += (size_t)surveys[k]->g.nf;
  }
  if (jobs > kStaticJobs)
    return fail(EHI_EINVAL, "batch of " + std::to_string(jobs) + " (survey, frequency) jobs exceeds the "
                            "static job table (" + std::to_string(kStaticJobs) + ")");
  void* table = nullptr;
  ehi_status st = scratch_for_current_device(&table);
  if (st != EHI_OK) return st;
  return factor_batch_impl(surveys, n, mu, table, sizeof(scratch), stream, bad_survey, bad_freq);
}

ehi_status ehi_hbm_probe(int32_t mode, const void* a, const void* b, void* c, void* d, void* e, size_t bytes,
                         double e_frac, int32_t grid, void* sink, void* stream) {
  g_err.clear();
  if (mode < 0 || mode > 4) return fail(EHI_EINVAL, "mode must be 0..4");
  if (bytes < 16 || bytes % 16 != 0) return fail(EHI_EINVAL, "bytes must be a positive multiple of 16");
  if (grid < 1 || grid > (1 << 20)) return fail(EHI_EINVAL, "grid must be in [1, 2^20]");
  if (!(e_frac >= 0.0 && e_frac <= 2.0)) return fail(EHI_EINVAL, "e_frac must be in [0, 2]");
  const bool two = mode >= 2;
  const int writes = mode == 0 ? 1 : mode == 2 ? 2 : mode == 3 ? 3 : 0;
  if (!a || (two && !b) || (writes >= 1 && !c) || (writes >= 2 && !d) || (writes >= 3 && !e) || (writes == 0 && !sink))
    return fail(EHI_EINVAL, "a buffer the mode uses is NULL");
  EHI_TRY(ehi::launch_stream_probe(mode, a, b, c, d, e, bytes, e_frac, grid, sink, static_cast<hipStream_t>(stream)),
          "hbm probe");
  return EHI_OK;
}

ehi_status ehi_set_refinement(ehi_survey* s, int32_t steps) {
  g_err.clear();
  if (!s) return fail(EHI_EINVAL, "survey is NULL");
  if (steps < 0 || steps > 4) return fail(EHI_EINVAL, "steps must be in [0, 4]");
  if (steps > 0 && s->precision != EHI_PREC_SPLIT_BF16)
    return fail(EHI_EINVAL, "refinement needs the FP64 factors of the split-BF16 form");
  s->refine = steps;
  return EHI_OK;
}

ehi_status ehi_set_stream(ehi_survey* s, void* stream) {
  g_err.clear();
  if (!s) return fail(EHI_EINVAL, "survey is NULL");
  PROF_END();
  s->stream = static_cast<hipStream_t>(stream);
  return EHI_OK;
}

ehi_status ehi_set_launch(ehi_survey* s, int32_t tblock, int32_t seg_rows, int32_t band) {
  g_err.clear();
  if (!s) return fail(EHI_EINVAL, "survey is NULL");
  if (tblock != 0 && tblock != 4 && tblock != 8) return fail(EHI_EINVAL, "tblock must be 0, 4 or 8");
  if (seg_rows != 0 && (seg_rows < ehi::kMinSegRows || seg_rows > ehi::kMaxSegRows))
    return fail(EHI_EINVAL, "seg_rows must be 0 or 16..512");
  if (band != -1 && band != 0 && band != 256 && band != 384 && band != 448 && band != 512)
    return fail(EHI_EINVAL, "band must be -1, 0, 256, 384, 448 or 512");
  if (tblock) s->g.tblock = tblock;
  if (seg_rows) s->g.seg_rows = seg_rows;
  if (band != -1) s->g.band_req = band;
  s->g.band = s->g.band_req ? s->g.band_req : ehi::march_band_for(s->g.X, s->g.tblock);
  return EHI_OK;
}

ehi_status ehi_get_launch(const ehi_survey* s, int32_t* tblock, int32_t* seg_rows, int32_t* band) {
  g_err.clear();
  if (!s) return fail(EHI_EINVAL, "survey is NULL");
  if (tblock) *tblock = s->g.tblock;
  if (seg_rows) *seg_rows = s->g.seg_rows;
  if (band) *band = s->g.band;
  return EHI_OK;
}

ehi_status ehi_apply_multipliers(ehi_survey* s, const void* resid_dev, void* mult_dev, int32_t ns,
                                 void* stream) {
  g_err.clear();
  if (!s) return fail(EHI_EINVAL, "survey is NULL");
  if (s->state < ehi::State::Factored) return fail(EHI_ESTATE, "apply before a successful factor");
  if (ns < 0) return fail(EHI_EINVAL, "ns must be >= 0");
  if (ns == 0) return EHI_OK;
  if (!resid_dev || !mult_dev) return fail(EHI_EINVAL, "residual or output is NULL");
  if (resid_dev == mult_dev) return fail(EHI_EINVAL, "residual and output may not alias");
  const ehi::Geometry& g = s->g;
  const ehi::Layout& L = s->L;
  hipStream_t st = stream ? static_cast<hipStream_t>(stream) : s->stream;
  const float2* R = static_cast<const float2*>(resid_dev);
  float2* X = static_cast<float2*>(mult_dev);
  double2* x64 = s->ptr<double2>(L.x64);
  PROF(EHI_PROF_SOLVE, st);
  const int refine = s->refine;
  for (int s0 = 0; s0 < ns; s0 += g.max_ns) {
    const int cnt = std::min(g.max_ns, ns - s0);
    EHI_TRY(ehi::launch_apply(g, s->ptr<float2>(L.m32), s->ptr<double2>(L.qhat), R, ns, s0, cnt,
                              refine, s->ptr<float2>(L.y32), s->ptr<float2>(L.r32), x64, X, st),
            "apply");
    PROF_N(2 + 3 * refine);
  }
  PROF_END();
  return EHI_OK;
}

ehi_status ehi_lambda_max(ehi_survey* s, double* out) {
  g_err.clear();
  if (!s || !out) return fail(EHI_EINVAL, "NULL argument");
  if (s->state < ehi::State::Hessian) return fail(EHI_ESTATE, "lambda_max before build_hessian");
  const ehi::Geometry& g = s->g;
  double* eig = s->ptr<double>(s->L.eig);
  EHI_TRY(ehi::launch_power_iter(g, s->ptr<double2>(s->L.hhat), eig, 400, s->stream), "power iteration");
  std::vector<double> host(g.nf);
  EHI_TRY(hipMemcpyAsync(host.data(), eig, sizeof(double) * g.nf, hipMemcpyDeviceToHost, s->stream),
          "eig readback");
  EHI_TRY(hipStreamSynchronize(s->stream), "lambda sync");
  *out = *std::max_element(host.begin(), host.end());
  return EHI_OK;
}

ehi_status ehi_copy_green_dft(ehi_survey* s, void* out_dev) {
  g_err.clear();
  if (!s || !out_dev) return fail(EHI_EINVAL, "NULL argument");
  if (s->state < ehi::State::Green) return fail(EHI_ESTATE, "no Green-function spectra yet");
  if (s->g.keep_z > 0)
    return fail(EHI_EINVAL, "a compressed survey holds the compressed spectra only (ehi_copy_compressed)");
  size_t bytes = sizeof(float2) * (size_t)s->g.nf * s->g.nr * s->g.nsub;
  EHI_TRY(hipMemcpyAsync(out_dev, s->ws + s->L.ghat, bytes, hipMemcpyDeviceToDevice, s->stream),
          "copy green");
  return EHI_OK;
}

ehi_status ehi_copy_compressed(ehi_survey* s, void* out_dev) {
  g_err.clear();
  if (!s || !out_dev) return fail(EHI_EINVAL, "NULL argument");
  if (s->g.keep_z <= 0) return fail(EHI_EINVAL, "the survey is not compressed");
  if (s->state < ehi::State::Green) return fail(EHI_ESTATE, "no Green-function spectra yet");
  size_t bytes = sizeof(float2) * (size_t)s->g.nf * s->g.nr * s->g.keep_z * s->g.keep_x;
  EHI_TRY(hipMemcpyAsync(out_dev, s->ws + s->L.gcomp, bytes, hipMemcpyDeviceToDevice, s->stream),
          "copy compressed");
  return EHI_OK;
}

ehi_status ehi_load_green_dft(ehi_survey* s, const void* in_dev) {
  g_err.clear();
  if (!s || !in_dev) return fail(EHI_EINVAL, "NULL argument");
  if (s->g.weighting == EHI_WEIGHT_FINITE_RECORD)
    return fail(EHI_ESTATE, "the finite-record weighting is built from the time samples (ehi_build_green)");
  const ehi::Geometry& g = s->g;
  if (g.keep_z > 0) {
    // straight into the compressed spectra, gh_rows receivers at a time
    const float2* in = static_cast<const float2*>(in_dev);
    for (int r0 = 0; r0 < g.nr; r0 += g.gh_rows) {
      const int nb_now = std::min(g.gh_rows, g.nr - r0);
      EHI_TRY(ehi::launch_dct_compress(g, in + (size_t)r0 * g.nsub, g.nr, r0, nb_now, s->ptr<float2>(s->L.dctz),
                                       s->ptr<float2>(s->L.dctx), s->ptr<float2>(s->L.dtmp),
                                       s->ptr<float2>(s->L.gcomp), s->stream),
              "spatial compression");
    }
    s->state = ehi::State::Green;
    return EHI_OK;
  }
  size_t bytes = sizeof(float2) * (size_t)g.nf * g.nr * g.nsub;
  EHI_TRY(hipMemcpyAsync(s->ws + s->L.ghat, in_dev, bytes, hipMemcpyDeviceToDevice, s->stream),
          "load green");
  s->state = ehi::State::Green;
  return EHI_OK;
}

ehi_status ehi_copy_hessian(ehi_survey* s, void* out_dev) {
  g_err.clear();
  if (!s || !out_dev) return fail(EHI_EINVAL, "NULL argument");
  if (s->state < ehi::State::Hessian) return fail(EHI_ESTATE, "no Hessian yet");
  size_t bytes = sizeof(double2) * (size_t)s->g.nf * s->g.nr * s->g.nr;
  EHI_TRY(hipMemcpyAsync(out_dev, s->ws + s->L.hhat, bytes, hipMemcpyDeviceToDevice, s->stream),
          "copy hessian");
  return EHI_OK;
}

ehi_status ehi_load_hessian(ehi_survey* s, const void* in_dev) {
  g_err.clear();
  if (!s || !in_dev) return fail(EHI_EINVAL, "NULL argument");
  size_t bytes = sizeof(double2) * (size_t)s->g.nf * s->g.nr * s->g.nr;
  EHI_TRY(hipMemcpyAsync(s->ws + s->L.hhat, in_dev, bytes, hipMemcpyDeviceToDevice, s->stream),
          "load hessian");
  s->state = ehi::State::Hessian;
  return EHI_OK;
}

ehi_status ehi_copy_factor(ehi_survey* s, void* out_dev) {
  g_err.clear();
  if (!s || !out_dev) return fail(EHI_EINVAL, "NULL argument");
  if (s->state < ehi::State::Factored) return fail(EHI_ESTATE, "no factor yet");
  const size_t nn = (size_t)s->g.nf * s->g.nr * s->g.nr;
  if (s->precision == EHI_PREC_SPLIT_BF16) {
    EHI_TRY(hipMemcpyAsync(out_dev, s->ws + s->L.lfac, sizeof(double2) * nn, hipMemcpyDeviceToDevice,
                           s->stream),
            "copy factor");
  } else {
    EHI_TRY(ehi::launch_c128_from_c64(s->ptr<float2>(s->L.lfac32), static_cast<double2*>(out_dev), nn,
                                      s->stream),
            "copy factor");
  }
  return EHI_OK;
}

ehi_status ehi_set_medium(ehi_survey* s, const float* vel_dev) {
  g_err.clear();
  if (!s) return fail(EHI_EINVAL, "survey is NULL");
  if (!vel_dev) return fail(EHI_EINVAL, "velocity is NULL");
  const ehi::Geometry& g = s->g;
  const ehi::Layout& L = s->L;
  hipStream_t st = s->stream;
  uint32_t* vmax = s->ptr<uint32_t>(L.vmax);
  PROF(EHI_PROF_SETUP, st);
  EHI_TRY(ehi::launch_vmax(vel_dev, g.nz * g.nx, vmax, st), "vmax");
  EHI_TRY(ehi::launch_coefficients(g, vel_dev, vmax, s->ptr<float>(L.ca), s->ptr<float>(L.bd), st),
          "coefficients");
  PROF_N(2);
  PROF_END();
  s->medium = true;
  return EHI_OK;
}

namespace {

// Shared checks of the modelling calls (the message is set on failure).
ehi_status model_check(ehi_survey* s, const void* in, const void* out, int32_t ns) {
  if (!s) return fail(EHI_EINVAL, "survey is NULL");
  if (!s->medium) return fail(EHI_ESTATE, "no medium: call build_green or set_medium first");
  if (ns < 0 || ns > (1 << 20)) return fail(EHI_EINVAL, "ns must be in [0, 2^20]");
  if (ns > 0 && (!in || !out)) return fail(EHI_EINVAL, "input or output is NULL");
  if (ns > 0 && in == out) return fail(EHI_EINVAL, "input and output may not alias");
  if (s->g.Z > 65535) return fail(EHI_EINVAL, "padded grid taller than 65535 rows");
  return EHI_OK;
}

}  // namespace

namespace {

// S (mode 1) or S^T (mode 2) on the marching kernel, 8 time levels per launch:
// needs distinct receiver cells and buffers the 32-bit buffer offsets reach.
bool march_model_ok(const ehi_survey* s) {
  const ehi::Geometry& g = s->g;
  return s->rec_distinct && g.tblock == 8 && (long long)g.nt * g.nsub * 4 < (1LL << 31) &&
         (long long)g.nr * g.nt * 4 < (1LL << 31);
}

ehi_status march_model(ehi_survey* s, int mode, const float* in, int32_t ns, float* out) {
  // segment height for about 1024 workgroups per launch (a modelling batch holds
  // fewer fields than a Green-function batch has receivers), 32 rows at least;
  // the Green-function build rebuilds its own row table
  ehi::Geometry g = s->g;
  {
    const int fields = std::min(g.nrb, ns);
    const int want_seg = ehi::cdiv(1024, std::max(1, fields * ehi::march_bands(g)));
    int seg = std::max(32, ehi::cdiv(ehi::cdiv(g.Z, want_seg), 16) * 16);
    if (const char* e = std::getenv("EHI_MODEL_SEG")) {
      const int v = std::atoi(e);
      if (v >= ehi::kMinSegRows && v <= ehi::kMaxSegRows) seg = v;
    }
    g.seg_rows = std::min(seg, ehi::kMaxSegRows);
  }
  const ehi::Layout& L = s->L;
  hipStream_t st = s->stream;
  const float* ca = s->ptr<float>(L.ca);
  const float* bd = s->ptr<float>(L.bd);
  ehi::RowEntry* rowtab = s->ptr<ehi::RowEntry>(L.rowtab);
  float* ub[2] = {s->ptr<float>(L.u0), s->ptr<float>(L.u1)};
  float* wb[2] = {s->ptr<float>(L.w0), s->ptr<float>(L.w1)};
  const size_t src_field = (size_t)g.nt * g.nsub, d_field = (size_t)g.nr * g.nt;
  PROF(EHI_PROF_MODEL, st);
  // the row table of the current launch shape (set_launch may have changed it)
  EHI_TRY(ehi::launch_row_table(g, bd, s->ptr<int32_t>(L.rowrec), rowtab, st), "row table");
  PROF_N(1);
  for (int s0 = 0; s0 < ns; s0 += g.nrb) {
    const int nb = std::min(g.nrb, ns - s0);
    const size_t nplane = (size_t)nb * g.plane();
    for (int b = 0; b < 2; ++b) {
      EHI_TRY(ehi::launch_fill_u32(reinterpret_cast<uint32_t*>(ub[b]), 0u, nplane, st), "fill");
      EHI_TRY(ehi::launch_fill_u32(reinterpret_cast<uint32_t*>(wb[b]), 0u, nplane, st), "fill");
    }
    PROF_N(4);
    ehi::ModelArgs m{};
    m.recmap = s->ptr<int32_t>(L.recmap);
    m.src_field = src_field;
    m.dat_field = d_field;
    m.sub_field = src_field;
    m.nt = g.nt;
    m.scale = (float)(12.0 * g.h * g.h);
    if (mode == 1) {
      m.src = in + (size_t)s0 * src_field;
      m.dat_out = out + (size_t)s0 * d_field;
    } else {
      m.dat_in = in + (size_t)s0 * d_field;
      m.sub_out = out + (size_t)s0 * src_field;
    }
    int cur = 0;
    for (int n = 0; n < g.nt; n += 8) {
      const int nlev = std::min(8, g.nt - n);
      m.n_in = n;
      EHI_TRY(ehi::launch_march_model(g, mode, ca, bd, rowtab, ub[cur], wb[cur], ub[1 - cur], wb[1 - cur], m,
                                      nlev, nb, st),
              mode == 1 ? "forward steps" : "adjoint steps");
      PROF_N(1);
      cur = 1 - cur;
    }
  }
  PROF_END();
  return EHI_OK;
}

}  // namespace

ehi_status ehi_forward_subgrid(ehi_survey* s, const float* src_dev, int32_t ns, float* data_dev) {
  g_err.clear();
  ehi_status chk = model_check(s, src_dev, data_dev, ns);
  if (chk != EHI_OK || ns == 0) return chk;
  if (march_model_ok(s)) return march_model(s, 1, src_dev, ns, data_dev);
  const ehi::Geometry& g = s->g;
  const ehi::Layout& L = s->L;
  hipStream_t st = s->stream;
  const float* ca = s->ptr<float>(L.ca);
  const float* bd = s->ptr<float>(L.bd);
  const int32_t* rec = s->ptr<int32_t>(L.rec);
  float* ub[2] = {s->ptr<float>(L.u0), s->ptr<float>(L.u1)};
  float* w = s->ptr<float>(L.w0);
  const size_t src_field = (size_t)g.nt * g.nsub, d_field = (size_t)g.nr * g.nt;
  PROF(EHI_PROF_MODEL, st);
  for (int s0 = 0; s0 < ns; s0 += g.nrb) {
    const int nb = std::min(g.nrb, ns - s0);
    const size_t nplane = (size_t)nb * g.plane();
    for (int b = 0; b < 2; ++b)
      EHI_TRY(ehi::launch_fill_u32(reinterpret_cast<uint32_t*>(ub[b]), 0u, nplane, st), "fill");
    EHI_TRY(ehi::launch_fill_u32(reinterpret_cast<uint32_t*>(w), 0u, nplane, st), "fill");
    PROF_N(3);
    const float* src = src_dev + (size_t)s0 * src_field;
    float* d = data_dev + (size_t)s0 * d_field;
    int cur = 0;
    for (int n = 0; n < g.nt; ++n) {
      // f^n enters u^{n+1}; trace sample n + 1 is stored at column n
      EHI_TRY(ehi::launch_fd_step(g, ca, bd, ub[cur], ub[1 - cur], w, nb, src + (size_t)n * g.nsub,
                                  src_field, st),
              "forward step");
      EHI_TRY(ehi::launch_record_points(g, rec, ub[1 - cur], d, d_field, n, nb, st), "record traces");
      PROF_N(2);
      cur = 1 - cur;
    }
  }
  PROF_END();
  return EHI_OK;
}

ehi_status ehi_backpropagate(ehi_survey* s, const float* data_dev, int32_t ns, float* src_dev) {
  g_err.clear();
  ehi_status chk = model_check(s, data_dev, src_dev, ns);
  if (chk != EHI_OK || ns == 0) return chk;
  if (march_model_ok(s)) return march_model(s, 2, data_dev, ns, src_dev);
  const ehi::Geometry& g = s->g;
  const ehi::Layout& L = s->L;
  hipStream_t st = s->stream;
  const float* ca = s->ptr<float>(L.ca);
  const float* bd = s->ptr<float>(L.bd);
  const int32_t* rec = s->ptr<int32_t>(L.rec);
  float* ub[2] = {s->ptr<float>(L.u0), s->ptr<float>(L.u1)};
  float* w = s->ptr<float>(L.w0);
  const size_t src_field = (size_t)g.nt * g.nsub, d_field = (size_t)g.nr * g.nt;
  PROF(EHI_PROF_MODEL, st);
  for (int s0 = 0; s0 < ns; s0 += g.nrb) {
    const int nb = std::min(g.nrb, ns - s0);
    const size_t nplane = (size_t)nb * g.plane();
    for (int b = 0; b < 2; ++b)
      EHI_TRY(ehi::launch_fill_u32(reinterpret_cast<uint32_t*>(ub[b]), 0u, nplane, st), "fill");
    EHI_TRY(ehi::launch_fill_u32(reinterpret_cast<uint32_t*>(w), 0u, nplane, st), "fill");
    PROF_N(3);
    const float* d = data_dev + (size_t)s0 * d_field;
    float* out = src_dev + (size_t)s0 * src_field;
    int cur = 0;
    for (int k = 0; k < g.nt; ++k) {
      // reversed time: step k injects trace sample nt - k (column nt - 1 - k);
      // u^{k+1} is the source-side field of step nt - 1 - k
      EHI_TRY(ehi::launch_fd_step(g, ca, bd, ub[cur], ub[1 - cur], w, nb, nullptr, 0, st), "adjoint step");
      EHI_TRY(ehi::launch_inject_points(g, ca, rec, d, d_field, g.nt - 1 - k, nb, ub[1 - cur], w, st),
              "inject traces");
      EHI_TRY(ehi::launch_record_subgrid(g, ub[1 - cur], out, src_field, g.nt - 1 - k, nb, st),
              "record subgrid");
      PROF_N(3);
      cur = 1 - cur;
    }
  }
  PROF_END();
  return EHI_OK;
}

ehi_status ehi_residual_spectra(ehi_survey* s, const float* dres_dev, int32_t ns, void* resid_dev,
                                void* stream) {
  g_err.clear();
  if (!s) return fail(EHI_EINVAL, "survey is NULL");
  if (ns < 0 || ns > (1 << 20)) return fail(EHI_EINVAL, "ns must be in [0, 2^20]");
  if (ns == 0) return EHI_OK;
  if (!dres_dev || !resid_dev) return fail(EHI_EINVAL, "input or output is NULL");
  const ehi::Geometry& g = s->g;
  hipStream_t st = stream ? static_cast<hipStream_t>(stream) : s->stream;
  PROF(EHI_PROF_MODEL, st);
  EHI_TRY(ehi::launch_resid_spectra(g, dres_dev, ns * g.nr, s->ptr<float2>(s->L.tw),
                                    static_cast<float2*>(resid_dev), st),
          "residual spectra");
  PROF_N(1);
  PROF_END();
  return EHI_OK;
}

ehi_status ehi_multipliers_to_time(ehi_survey* s, const void* mult_dev, int32_t ns, float* out_dev,
                                   void* stream) {
  g_err.clear();
  if (!s) return fail(EHI_EINVAL, "survey is NULL");
  if (ns < 0 || ns > (1 << 20)) return fail(EHI_EINVAL, "ns must be in [0, 2^20]");
  const ehi::Geometry& g = s->g;
  // the frequencies must be distinct bins 0..nt of the 2nt-point transform
  unsigned long long edge = 0;
  std::vector<long long> seen;
  for (int f = 0; f < g.nf; ++f) {
    const double k = s->freq[f] * 2.0 * g.nt * g.dt;
    const double kr = std::nearbyint(k);
    if (std::fabs(k - kr) > 1e-6 || kr < 0 || kr > g.nt)
      return fail(EHI_EINVAL, "frequencies are not bins 0..nt of the 2nt-point transform");
    const long long ki = (long long)kr;
    if (std::find(seen.begin(), seen.end(), ki) != seen.end())
      return fail(EHI_EINVAL, "a frequency bin occurs twice");
    seen.push_back(ki);
    if (ki == 0 || ki == g.nt) edge |= 1ull << f;
  }
  if (ns == 0) return EHI_OK;
  if (!mult_dev || !out_dev) return fail(EHI_EINVAL, "input or output is NULL");
  if (g.nt > 65535 * 64) return fail(EHI_EINVAL, "nt too large for the inverse transform");
  hipStream_t st = stream ? static_cast<hipStream_t>(stream) : s->stream;
  PROF(EHI_PROF_MODEL, st);
  EHI_TRY(ehi::launch_to_time(g, static_cast<const float2*>(mult_dev), ns * g.nr, s->ptr<float2>(s->L.tw),
                              edge, out_dev, st),
          "inverse transform");
  PROF_N(1);
  PROF_END();
  return EHI_OK;
}

ehi_status ehi_misfit(const float* dd_dev, const float* pred_dev, const float* obs_dev, int32_t ns,
                      int64_t len, float* err_dev, double* relerr_dev, void* stream) {
  g_err.clear();
  if (ns < 0 || len < 1) return fail(EHI_EINVAL, "need ns >= 0 and len >= 1");
  if (ns == 0) return EHI_OK;
  if (!dd_dev || !pred_dev || !obs_dev || !relerr_dev) return fail(EHI_EINVAL, "NULL argument");
  EHI_TRY(ehi::launch_misfit(dd_dev, pred_dev, obs_dev, ns, (size_t)len, err_dev, relerr_dev,
                             static_cast<hipStream_t>(stream)),
          "misfit");
  return EHI_OK;
}

namespace {

ehi_status cg_check(int32_t ns, int64_t len, std::initializer_list<const void*> ptrs) {
  if (ns < 0 || len < 1) return fail(EHI_EINVAL, "need ns >= 0 and len >= 1");
  if (ns > 0)
    for (const void* q : ptrs)
      if (!q) return fail(EHI_EINVAL, "NULL argument");
  return EHI_OK;
}

}  // namespace

ehi_status ehi_cg_init(const float* dd_dev, int32_t ns, int64_t len, float* x_dev, float* r_dev,
                       float* p_dev, double* rr_dev, void* stream) {
  g_err.clear();
  ehi_status c = cg_check(ns, len, {dd_dev, x_dev, r_dev, p_dev, rr_dev});
  if (c != EHI_OK || ns == 0) return c;
  EHI_TRY(ehi::launch_cg_init(dd_dev, x_dev, r_dev, p_dev, ns, (size_t)len, rr_dev,
                              static_cast<hipStream_t>(stream)),
          "cg init");
  return EHI_OK;
}

ehi_status ehi_cg_shift_dot(float* ap_dev, const float* p_dev, double mu, int32_t ns, int64_t len,
                            double* pap_dev, void* stream) {
  g_err.clear();
  ehi_status c = cg_check(ns, len, {ap_dev, p_dev, pap_dev});
  if (c != EHI_OK || ns == 0) return c;
  EHI_TRY(ehi::launch_cg_shift_dot(ap_dev, p_dev, (float)mu, ns, (size_t)len, pap_dev,
                                   static_cast<hipStream_t>(stream)),
          "cg shift");
  return EHI_OK;
}

ehi_status ehi_cg_update(float* x_dev, float* r_dev, const float* p_dev, const float* ap_dev,
                         const double* rr_dev, const double* pap_dev, double mu, int32_t ns, int64_t len,
                         double* rr_new_dev, double* fit_dev, void* stream) {
  g_err.clear();
  ehi_status c = cg_check(ns, len, {x_dev, r_dev, p_dev, ap_dev, rr_dev, pap_dev, rr_new_dev, fit_dev});
  if (c != EHI_OK || ns == 0) return c;
  EHI_TRY(ehi::launch_cg_update(x_dev, r_dev, p_dev, ap_dev, rr_dev, pap_dev, (float)mu, ns, (size_t)len,
                                rr_new_dev, fit_dev, static_cast<hipStream_t>(stream)),
          "cg update");
  return EHI_OK;
}

ehi_status ehi_cg_direction(float* p_dev, const float* r_dev, const double* rr_new_dev, const double* rr_dev,
                            int32_t ns, int64_t len, void* stream) {
  g_err.clear();
  ehi_status c = cg_check(ns, len, {p_dev, r_dev, rr_new_dev, rr_dev});
  if (c != EHI_OK || ns == 0) return c;
  EHI_TRY(ehi::launch_cg_direction(p_dev, r_dev, rr_new_dev, rr_dev, ns, (size_t)len,
                                   static_cast<hipStream_t>(stream)),
          "cg direction");
  return EHI_OK;
}

ehi_status ehi_mdot(const float* v_dev, int64_t vstride, int32_t nvec, const float* w_dev, int32_t ns,
                    int64_t len, double* out_dev, void* stream) {
  g_err.clear();
  if (nvec < 0 || nvec > 65535 || ns > 65535) return fail(EHI_EINVAL, "nvec and ns must be in [0, 65535]");
  ehi_status c = cg_check(ns, len, {v_dev, w_dev, out_dev});
  if (c != EHI_OK || ns == 0 || nvec == 0) return c;
  if (vstride < len) return fail(EHI_EINVAL, "vstride must be >= len");
  EHI_TRY(ehi::launch_mdot(v_dev, (size_t)vstride, nvec, w_dev, ns, (size_t)len, out_dev,
                           static_cast<hipStream_t>(stream)),
          "mdot");
  return EHI_OK;
}

ehi_status ehi_combine(const float* v_dev, int64_t vstride, int32_t nvec, const double* coef_dev, int32_t ns,
                       int64_t len, double beta, float* dst_dev, void* stream) {
  g_err.clear();
  if (nvec < 0 || nvec > 1024 || ns > 65535) return fail(EHI_EINVAL, "nvec must be in [0, 1024], ns <= 65535");
  ehi_status c = cg_check(ns, len, {v_dev, coef_dev, dst_dev});
  if (c != EHI_OK || ns == 0) return c;
  if (nvec > 0 && vstride < len) return fail(EHI_EINVAL, "vstride must be >= len");
  EHI_TRY(ehi::launch_combine(v_dev, (size_t)vstride, nvec, coef_dev, ns, (size_t)len, beta, dst_dev,
                              static_cast<hipStream_t>(stream)),
          "combine");
  return EHI_OK;
}

}  // extern "C"
