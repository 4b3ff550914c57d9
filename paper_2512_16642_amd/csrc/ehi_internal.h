// Internal declarations of libehi: workspace layout, survey state, launchers.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

#include "../../include/ehi.h"

namespace ehi {

// ---- fixed design constants -------------------------------------------------
constexpr int kGhost = 2;        // zero ring around the padded grid (stencil radius)
constexpr int kRowAlign = 64;    // padded row pitch is a multiple of 64 floats (256 B)
constexpr int kMaxSponge = 512;  // largest absorbing-layer width (cells)
constexpr int kHerkTile = 32;    // Hessian output tile (rows = cols)
constexpr int kHerkSplitMax = 64;  // max split-K partitions of the grid sum
// Default partitions hold at most this many 32-point stages: each partition
// adds its stages into FP32 running sums, whose rounding error grows about
// linearly with the number of stages added, and the low-frequency systems
// amplify that error in the multipliers (partial sums are combined in FP64).
constexpr int kHerkMaxStages = 40;
constexpr size_t kAlign = 256;
constexpr int kMaxDecim = 64;    // largest time-axis resampling factor
constexpr int kMaxDecimK = 512;  // largest half-length of its low-pass filter

__host__ __device__ inline size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }
__host__ __device__ inline int cdiv(int a, int b) { return (a + b - 1) / b; }

// Geometry derived from the descriptor.
struct Geometry {
  int nz, nx, nb;
  int Z, X;        // padded grid (interior + absorbing layer)
  int Zp, Xp;      // allocated plane incl. ghost ring and row padding
  int stride, sshift, nzs, nxs, nsub;  // stride = 1 << sshift
  int nsub_p;      // staging row pitch (nsub rounded up to 256)
  int chunk;       // time samples per DFT chunk (staging depth; multiple of 4 and tblock)
  int windows;     // staging windows: 1, or 2 (the DFT of one overlaps the stepping of the next)
  int nt, nr, nf, nrb, max_ns;
  int herk_split;  // split-K partitions
  int herk_whole;  // 1: one workgroup per (frequency, partition) forms all of Hhat (nr <= 224)
  int herk_form;   // descriptor request: 0 auto, 1 whole-matrix, 2 tile pairs, 3 plain form on vector units
  int split_bf16;  // 1: split-BF16 contraction, 0: plain FP32
  int weighting;   // EHI_WEIGHT_LONG_RECORD or EHI_WEIGHT_FINITE_RECORD
  int keep_z, keep_x;  // leading DCT-II coefficients kept along z and x of the subgrid (0 = no transform)
  int gh_rows;     // receivers per frequency held in the spectra buffer: nr, or nrb when compressed
  int dft_form;    // 0: FP32 matrix-core DFT; 1: three-part BF16 split on the BF16 matrix cores (default)
  // time-axis resampling of the finite-record weighting (decim = 1: every sample)
  int decim;       // D: every D-th filtered sample is kept
  int dK;          // filter half-length (taps j = -dK..dK)
  int dM;          // kept samples: n_q = 1 - dK + q D, q = 0..dM-1 (support meets the record)
  int dqa, dqb;    // kept samples inside the record (1 <= n_q <= nt): q in [dqa, dqb]
  int dhist;       // samples of the previous window kept for the filter (2 dK)
  int drows;       // rows of the kept-sample buffer per receiver (most kept samples one window yields)
  int tblock;      // time levels per marching launch (2, 4 or 8; divides chunk)
  int seg_rows;    // output rows per marching segment
  int band;        // columns per marching workgroup (256, 384, 448 or 512)
  int band_req;    // requested band width, 0 = the one with the fewest lanes for tblock
  double h, dt;
  __host__ __device__ size_t plane() const { return (size_t)Zp * Xp; }
};

// Byte offsets of every buffer inside the caller's workspace.
struct Layout {
  size_t freq;      // double [nf]
  size_t rec;       // int32 [2][nr]  (iz then ix, interior indices)
  size_t ca;        // float [Zp][Xp]  kappa / (12 h^2 a)
  size_t bd;        // float [kMaxSponge + 1]  b / a by distance into the layer
  size_t rowtab;    // RowEntry [cdiv(Z, kMinSegRows)][kRowTabStride]  marching row table
  size_t rowrec;    // int32 [Z]  1 if the padded row holds a receiver
  size_t recmap;    // int32 [Zp][Xp]  receiver index per cell (-1: none), for the modelling runs
  size_t vmax;      // uint32 [4]  max velocity bits
  size_t tw;        // float2 [nt][nf] exp(-i w n dt), n = 1..nt
  size_t u0, u1;    // float [nrb][Zp][Xp]  (ping-pong)
  size_t w0, w1;    // float [nrb][Zp][Xp]  (ping-pong)
  size_t stage;     // float [windows][nrb][chunk][nsub_p]
  size_t ghat;      // float2 [nf][gh_rows][nsub]  (compressed: one receiver batch's spectra)
  size_t hpart;     // float2 [split][nf][nr][nr]
  size_t hpart64;   // double2 [split][nf][nr][nr]  finite-record partial sums (else empty)
  size_t r2scale;   // double [nf]  finite-record Gram scale: 1/nt, or (D / H(w))^2 D / nt when resampled
  size_t gscale;    // double [nf]  D / H(w): the resampled running spectra to the record's spectra
  size_t dtaps;     // float [2 dK + 1]  resampling filter
  size_t dtw;       // float2 [dM][nf]  exp(-i w n_q dt) at the kept samples
  size_t dhistbuf;  // float [nrb][dhist][nsub_p]  last samples of the previous window
  size_t ddec;      // float [nrb][drows][nsub_p]  kept (filtered) samples of the current window
  size_t dctz, dctx;  // complex64 [keep_z][nzs], [keep_x][nxs] DCT-II rows (compression only)
  size_t dtmp;      // complex64 [nf][gh_rows][nxs][keep_z]  first pass of the 2D transform
  size_t gcomp;     // complex64 [nf][nr][keep_z * keep_x]  compressed spectra
  size_t hhat;      // double2 [nf][nr][nr]
  size_t qhat;      // double2 [nf][nr][nr]   Hhat + mu I (Hermitian, full)
  size_t lfac;      // double2 [nf][nr][nr]   lower Cholesky factor (FP64 mode)
  size_t lfac32;    // float2 [nf][nr][nr]    complex64 copy (or the FP32 factor)
  size_t m64;       // double2 [nf][np][np]  FP64 scratch of the triangular inverse
  size_t m32;       // float2 [nf][np][np]  complex64 M = L^{-1} (np = 32 cdiv(nr, 32))
  size_t y32;       // float2 [nf][max_ns][nr]  solve scratch
  size_t r32;       // float2 [nf][max_ns][nr]  refinement residual
  size_t x64;       // double2 [nf][max_ns][nr] refinement accumulator
  size_t status;    // int32 [nf + 4]
  size_t eig;       // double [nf]
  size_t jobs;      // FactorJob [nf]
  size_t total;
};

enum class State : int { Created = 0, Green = 1, Hessian = 2, Factored = 3 };

// One (survey, frequency) factorisation: pointers into that survey's workspace.
struct FactorJob {
  const double2* hhat;
  double2* qhat;
  double2* lfac;
  float2* l32;
  double2* m64;   // [np][np] FP64 scratch of the triangular inverse (np = 32 cdiv(nr, 32))
  float2* m32;    // [np][np] complex64 inverse M = L^{-1}, zero above the diagonal
  int32_t* status;
  double mu;
  int nr;
  int fp64;
};

// Event pairs bracketing runs of launches of one kind (EHI_PROF_*).
struct ProfRecord {
  int kind;
  int launches;
  hipEvent_t start, stop;
};

struct Profiler {
  bool on = false;
  std::vector<ProfRecord> recs;
  int open_kind = -1;
  int open_launches = 0;
  hipEvent_t open_start = nullptr;
  hipStream_t open_stream = nullptr;
  // start a run of `kind` on stream st (closes a run of another kind first)
  hipError_t begin(int kind, hipStream_t st);
  void count(int n = 1) { open_launches += n; }
  hipError_t end();
};

}  // namespace ehi

struct ehi_survey {
  ehi::Geometry g;
  ehi::Layout L;
  int precision;
  std::vector<int32_t> rec_iz, rec_ix;
  std::vector<double> freq;
  char* ws;
  size_t ws_bytes;
  hipStream_t stream;
  // two staging windows: the DFT (and finite-record contraction) of a window
  // runs on `side` while `stream` steps into the other window
  hipStream_t side;
  hipEvent_t ev_marched[2], ev_dft[2];
  int device;
  ehi::State state;
  bool medium;      // ca, bd hold a velocity model (build_green or set_medium)
  bool rec_distinct; // no two receivers share a cell (the marching modelling path applies)
  double mu;
  int refine;       // FP64-residual refinement steps of each deblur
  ehi::Profiler prof;
  template <class T>
  T* ptr(size_t off) const { return reinterpret_cast<T*>(ws + off); }
};

namespace ehi {

// Marching segments hold kMinSegRows..kMaxSegRows output rows.  A launch reads,
// per segment, kRowTabStride row-table entries: entry ti describes padded row
// z0 - 4T + ti (z0 = first owned row, T = time levels per launch).
constexpr int kMinSegRows = 16;
constexpr int kMaxSegRows = 512;
constexpr int kRowTabStride = kMaxSegRows + 6 * 8 + 8;

// bz = b / a of the row's distance into the top/bottom layer (1 outside the
// grid); own = byte offset of the row in a plane if the segment owns it, else
// -1; sub = byte offset of the row's subgrid line inside a staging slot if the
// segment owns it and it lies on the subgrid, else -1.  For the modelling
// runs: suball = the subgrid line offset for any row on the subgrid (owned or
// halo), recall = the row's byte offset in the receiver map for any row
// holding a receiver, recown = the same for owned rows only (else -1).
struct alignas(16) RowEntry {
  float bz;
  int32_t own, sub, recown;
  int32_t suball, recall, pad0, pad1;
};

// Arguments of the modelling modes of the marching kernel (forward S with a
// subgrid source and traces recorded at the receivers; S^T with the traces
// injected at the receivers and the field recorded on the subgrid).  Pointers
// are the batch's first field; field k adds k * the *_field strides (floats).
struct ModelArgs {
  const float* src;       // S: source [field][nt][nsub]
  const float* dat_in;    // S^T: traces [field][nr][nt]
  float* dat_out;         // S: traces [field][nr][nt]
  float* sub_out;         // S^T: subgrid field [field][nt][nsub]
  const int32_t* recmap;  // receiver index of every plane cell, -1 elsewhere
  size_t src_field, dat_field, sub_field;
  int n_in;               // sample index of the launch's input level
  int nt;
  float scale;            // 12 h^2: kappa f / a = ca 12 h^2 f
};

// ---- launchers (each returns hipGetLastError() of its launch) ----------------
hipError_t launch_fill_u32(uint32_t* p, uint32_t value, size_t n, hipStream_t st);
hipError_t launch_vmax(const float* vel, int n, uint32_t* out_bits, hipStream_t st);
hipError_t launch_coefficients(const Geometry& g, const float* vel, const uint32_t* vmax_bits,
                               float* ca, float* bd, hipStream_t st);
hipError_t launch_twiddles(const Geometry& g, const double* freq, float2* tw, hipStream_t st);
// zero the row padding [nsub, nsub_p) of every staging slot of every window
hipError_t launch_zero_stage_tails(const Geometry& g, float* stage, hipStream_t st);
hipError_t launch_wave_init(const Geometry& g, const float* vel, const int32_t* rec, int r0,
                            int nrb_now, float* u0, float* w0, float* stage, hipStream_t st);
int march_bands(const Geometry& g);
int march_band_for(int X, int tblock);  // band width covering X columns with the fewest lanes
hipError_t launch_row_table(const Geometry& g, const float* bd, const int32_t* rowrec, RowEntry* rt,
                            hipStream_t st);
// modelling runs on the marching kernel: mode 1 = S, mode 2 = S^T (tblock 8 only)
hipError_t launch_march_model(const Geometry& g, int mode, const float* ca, const float* bd, const RowEntry* rt,
                              const float* uin, const float* win, float* uout, float* wout,
                              const ModelArgs& m, int nlev, int nrb_now, hipStream_t st);
hipError_t launch_march(const Geometry& g, const float* ca, const float* bd, const RowEntry* rt,
                        const float* uin, const float* win, float* uout, float* wout, float* stage,
                        int slot0, int nlev, int nrb_now, hipStream_t st);
hipError_t launch_dft_chunk(const Geometry& g, const float* stage, const float2* tw, int n0,
                            int cnt, bool first, int r0, int nrb_now, float2* ghat,
                            hipStream_t st);
hipError_t launch_herk_fp32(const Geometry& g, const float2* ghat, float2* hpart, hipStream_t st);
hipError_t launch_herk_split_bf16(const Geometry& g, const float2* ghat, float2* hpart,
                                  hipStream_t st);
// the Gram of the running spectra enters the sums for steps gram_lo..gram_hi
// of the launch (every step without resampling)
hipError_t launch_herk_r2_chunk(const Geometry& g, const float* stage, const float2* tw,
                                const float2* ghat, int n0, int cnt, bool first, int gram_lo, int gram_hi,
                                double2* hpart64, hipStream_t st);
hipError_t launch_herk_r2_reduce(const Geometry& g, const double2* hpart64, const double* scale, double2* hhat,
                                 hipStream_t st);
// time-axis resampling (finite-record weighting)
hipError_t launch_decimate(const Geometry& g, const float* stage, const float* hist, const float* taps, int q0,
                           int cnt, int n_w0, int n_end, int nrb_now, float* dec, hipStream_t st);
hipError_t launch_hist_copy(const Geometry& g, const float* stage, int n_end, int nrb_now, float* hist,
                            hipStream_t st);
hipError_t launch_twiddles_at(int count, int nf, double dt, const double* freq, int n_first, int n_step,
                              float2* tw, hipStream_t st);
hipError_t launch_scale_spectra(const Geometry& g, const double* scale, float2* ghat, hipStream_t st);
hipError_t launch_dct_matrix(int n, int keep, float2* d, hipStream_t st);
// compressed spectra of nrows receivers: input rows f * rows_per_f + i, output
// rows f * nr + row0 + i of gcomp (tmp: [nf][nrows][nxs][keep_z])
hipError_t launch_dct_compress(const Geometry& g, const float2* ghat, int rows_per_f, int row0, int nrows,
                               const float2* dz, const float2* dx, float2* tmp, float2* gcomp, hipStream_t st);
hipError_t launch_herk_reduce(const Geometry& g, const float2* hpart, double2* hhat,
                              hipStream_t st);
int herk_whole_groups(int nr);  // workgroups per (frequency, partition) of the whole-matrix contraction
hipError_t launch_herk_compressed(const Geometry& g, const float2* gcomp, int K, double2* hhat,
                                  hipStream_t st);
hipError_t launch_factor_jobs(const FactorJob* jobs, int njobs, hipStream_t st);
hipError_t launch_minv_jobs(const FactorJob* jobs, int njobs, int max_nr, hipStream_t st);
int solve_blocks(const Geometry& g);
hipError_t launch_apply(const Geometry& g, const float2* m32, const double2* qhat, const float2* R,
                        int rld, int s0, int cnt, int refine, float2* y32, float2* r32,
                        double2* x64, float2* out, hipStream_t st);
hipError_t launch_power_iter(const Geometry& g, const double2* hhat, double* eig, int iters,
                             hipStream_t st);
hipError_t launch_c128_from_c64(const float2* in, double2* out, size_t n, hipStream_t st);
// forward modelling (S, S^T on the subgrid sources) and the time/frequency transfer
hipError_t launch_fd_step(const Geometry& g, const float* ca, const float* bd, const float* uin,
                          float* uout, float* w, int nb_now, const float* src, size_t src_field,
                          hipStream_t st);
hipError_t launch_inject_points(const Geometry& g, const float* ca, const int32_t* rec, const float* data,
                                size_t data_field, int col, int nb_now, float* uout, float* w,
                                hipStream_t st);
hipError_t launch_record_subgrid(const Geometry& g, const float* u, float* dst, size_t dst_field, int slot,
                                 int nb_now, hipStream_t st);
hipError_t launch_record_points(const Geometry& g, const int32_t* rec, const float* u, float* d,
                                size_t d_field, int col, int nb_now, hipStream_t st);
hipError_t launch_resid_spectra(const Geometry& g, const float* dres, int nq, const float2* tw, float2* R,
                                hipStream_t st);
hipError_t launch_to_time(const Geometry& g, const float2* X, int nq, const float2* tw,
                          unsigned long long edge_bins, float* x, hipStream_t st);
hipError_t launch_misfit(const float* dd, const float* pred, const float* obs, int ns, size_t len,
                         float* err, double* relerr, hipStream_t st);
hipError_t launch_mdot(const float* v, size_t vstride, int nvec, const float* w, int ns, size_t len,
                       double* out, hipStream_t st);
hipError_t launch_combine(const float* v, size_t vstride, int nvec, const double* coef, int ns, size_t len,
                          double beta, float* dst, hipStream_t st);
hipError_t launch_cg_init(const float* dd, float* x, float* r, float* p, int ns, size_t len, double* rr,
                          hipStream_t st);
hipError_t launch_cg_shift_dot(float* Ap, const float* p, float mu, int ns, size_t len, double* pAp,
                               hipStream_t st);
hipError_t launch_cg_update(float* x, float* r, const float* p, const float* Ap, const double* rr,
                            const double* pAp, float mu, int ns, size_t len, double* rr_new, double* fit,
                            hipStream_t st);
hipError_t launch_cg_direction(float* p, const float* r, const double* rr_new, const double* rr, int ns,
                               size_t len, hipStream_t st);
hipError_t launch_c64_from_c128(const double2* in, float2* out, size_t n, hipStream_t st);
hipError_t launch_stream_probe(int mode, const void* a, const void* b, void* c, void* d, void* e, size_t bytes,
                               double e_frac, int grid, void* sink, hipStream_t st);

}  // namespace ehi
