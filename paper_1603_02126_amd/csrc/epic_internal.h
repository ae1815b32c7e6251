// Internal interface between the host side of the library (plans, argument
// checks, dispatch) and the HIP kernels.  Not part of the public ABI.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace epic {

// Packed sample formats (same values as epic_efmt).
enum : int { kCF32 = 0, kCI8 = 1, kCI4 = 2 };

__host__ __device__ inline int efmt_bytes(int fmt) { return fmt == kCF32 ? 8 : fmt == kCI8 ? 2 : 1; }

// Hold bits per (channel, antenna), precomputed on the host.
enum : uint8_t { kHoldFlagged = 1, kHoldDZero = 2 };

// Fused imaging: calibrate + grid + 2D transform + |X|^2 accumulation over a
// range of samples, one partial image per (split, channel).
struct ImageArgs {
  const uint8_t* efield;    // [T][F][Na] packed
  int64_t n_t;              // samples processed (t = 0 .. n_t-1)
  int F, Na, fmt;
  const float2* u;          // [n_int][F][Na]: u of interval t / t_cal
  int64_t t_cal;
  const uint2* slots;       // gridding schedule [n_slots][lanes]
  int n_slots;
  int splits;               // workgroups per channel
  float* partial;           // [splits][F][N*N]
  // schedule of the half-frame gridding (64 lanes): columns 0..31, then
  // columns 32..63; for 64 x 64 the cell offsets are re-based to column 0 of
  // a kHalfPitch buffer, for the residue-class engines the codes keep the
  // sub-cell (the kernel re-bases); null when not built
  const uint2* slots_h = nullptr;
  int n_slots_h0 = 0, n_slots_h1 = 0;
  // snapshot form: one image per window of t_acc samples, written to
  // snap[window][F][N*N] scaled by snap_scale / (samples in the window);
  // splits then divide the windows of a channel (0: whole-run average)
  int64_t t_acc = 0;
  float* snap = nullptr;
  double snap_scale = 0.0;
  // multi-class schedules of the dense residue-class engine (N = 128, 256):
  // per half of the sub-cell columns, rows of 64 x (classes per frame) sub-cell
  // owners; null when not built
  const uint2* slots_m = nullptr;
  int n_slots_m0 = 0, n_slots_m1 = 0;
  // DFT-GEMM form: operand precision (0 fp16 hi + lo, 1 bf16 hi + lo, 2 bf16
  // hi + mid + lo) and, for N = 128, 256, its class schedule (128 owners, all
  // sub-cell columns, the dense engine's slot format)
  int dft_prec = 0;
  const uint2* slots_c = nullptr;
  int n_slots_c = 0;
  // residue-class engine choice at 128 / 256 with integer samples: 0 = the
  // default (class-pair engine where it applies, else the dense engine with
  // gridding batches of 2); 2 or 4 = the dense engine with that batch
  int grid_batch = 0;
};

// Stage-wise gridding to HBM.
struct GridArgs {
  const uint8_t* efield;
  int64_t t0;
  int nt, F, Na, fmt;
  const float2* u;          // [F][Na]
  const uint2* slots;
  int n_slots;
  float2* grid;             // [nt][F][N][N]
};

// Stage-wise transform + accumulate from HBM grids.
struct ImageAccArgs {
  const float2* grid;       // [nt][F][N][N]
  int nt, F;
  float inv_na;             // 1 / Na
  float* image;             // [F][N][N] +=
  float2* tap;              // [nt][F] or null
  const int* k0;            // [F][2] (kx, ky)
};

// EPICal solve over all intervals (fast path).
struct SolveArgs {
  const uint8_t* efield;
  int64_t n_t;
  int F, Na, fmt;
  int64_t t_cal;
  int n_int;
  const double2* A;         // [n_pix][F][Na]
  const double2* D;         // [n_pix][F][Na]
  const uint8_t* hold;      // [F][Na] kHold* bits
  double na_eff, gamma;
  double2* gains;           // [F][Na] in/out
  float2* u_hist;           // [n_int][F][Na] (written by launch_hist_to_u from g_hist)
  double2* g_hist;          // [n_int+1][F][Na], required
  uint32_t* status;         // [F][Na] or null
  int n_pix = 1;            // tapped pixels (1..kMaxPix; > 1 needs Na <= kSolveThreads)
};
constexpr int kMaxPix = 4;

// Gains shared over a band of channels.  Band model per antenna: mean mode
// (re, im); poly mode 4 amplitude and 4 phase coefficients (increasing
// powers of x).  NaN in slot 0: no model.
constexpr int kBandCoef = 8;
constexpr int kBandMaxDeg = 3;
enum : int { kBandNone = 0, kBandMean = 1, kBandPoly = 2 };

struct BandArgs {
  SolveArgs s;
  int b0, b1;               // band channels [b0, b1)
  int mode, deg_amp, deg_phase;
  const double* x;          // [F] band coordinate in [-1, 1] (band channels)
  double2* raw;             // [F][Na] undamped solutions of the current interval (NaN: none)
  double* coef;             // [Na][kBandCoef] band model of the current interval
  uint32_t* bar;            // grid barrier flags, one per workgroup (256), zero at launch
};

// Stage-wise EPICal accumulate / finalize.
struct UpdateArgs {
  const uint8_t* efield;
  int64_t t0;
  int nt, F, Na, fmt;
  const float2* tap;        // [nt][F]
  double* kq;               // [F][Na][4]
  double2* gains;
  const double2* A;
  const double2* D;
  const uint8_t* hold;
  double na_eff, gamma;
  int finalize;
  uint32_t* status;
};

// Adjoint of fixed-gain imaging.
struct AdjointArgs {
  const uint8_t* efield;
  int64_t n_t;
  int F, Na, fmt;
  const float2* u;          // [F][Na]
  const float* R;           // [F][N][N] dL/dI
  const uint2* slots;
  int n_slots;
  const uint32_t* cell_ixy; // [Na][K2]
  const float* cell_w;
  int k2;
  int splits;
  double2* partial;         // [splits][F][Na]
  // half-frame schedules (64 x 64 two-waves-per-SIMD engine), as in ImageArgs
  const uint2* slots_h = nullptr;
  int n_slots_h0 = 0, n_slots_h1 = 0;
};

// Batched execution over several arrays (one launch per stage).
constexpr int kMaxBatch = 16;

struct BatchImageArgs {
  ImageArgs arr[kMaxBatch];
  int code[kMaxBatch];      // body of each array (batch_body)
  int n_arrays;
  const int4* items;        // {array, channel, class group, split}, largest first
  int n_items;
  int* counter;             // work-queue head (reset by the launcher)
};

struct BatchSolveArgs {
  SolveArgs arr[kMaxBatch];
  int chan_off[kMaxBatch + 1];   // prefix sums of channel counts
  int n_arrays;
};

struct BatchReduceArgs {
  const float* partial[kMaxBatch];
  float* image[kMaxBatch];
  int splits[kMaxBatch];
  int64_t per_split[kMaxBatch];
  double scale[kMaxBatch];
  int64_t off[kMaxBatch + 1];
  int n_arrays;
  const int* error = nullptr;   // nonzero: the images are not valid (written as NaN)
};

// One launch for the calibration solve and the imaging of every array.  The
// first workgroups to start take the solve tasks (one channel each), publish
// each interval's FP32 u = 1/g as soon as it is known and raise the
// channel's progress counter; every workgroup then pulls imaging items, each
// waiting until the intervals its samples fall in are published.  A solve
// never waits, and every solve task is taken before any workgroup images, so
// the waits always end; each is bounded all the same and, if it runs out,
// sets *error (the reduction then writes NaN images).
// The solve fields that the array's ImageArgs does not already carry:
struct FusedSolveExtra {
  const double2* A;
  const double2* D;
  const uint8_t* hold;
  double2* gains;
  double2* g_hist;
  uint32_t* status;
  double na_eff, gamma;
  int n_int;
  int code;                 // 100 J + PS of the single-pixel solve body, kFusedMultiCode + PS with several pixels
  int n_pix;                // tapped pixels
};
constexpr int kFusedMultiCode = 1000;

struct FusedArgs {
  FusedSolveExtra sx[kMaxBatch];
  int chan_off[kMaxBatch + 1];   // prefix sums of channel counts: solve task -> (array, channel)
  int n_solve;
  int* ticket;              // role counter (reset by the launcher)
  int* progress;            // [n_solve] intervals published per channel (reset by the launcher)
  int* error;
  int max_polls;            // bound of one wait (kFusedWaitPolls unless set for a test)
};

hipError_t launch_run_fused(const BatchImageArgs& b, const FusedArgs& fa, int n_workgroups, hipStream_t s);
// the spin limit of one wait (polls of about 0.2 us each)
constexpr int kFusedWaitPolls = 1 << 23;

// Body of the persistent batched imaging kernel for an array (0: none, the
// array is imaged by its own launch in the batched sequence).
int batch_body(const ImageArgs& a, int N, bool dft);
hipError_t launch_image_batch(const BatchImageArgs& b, int n_workgroups, hipStream_t s);
hipError_t launch_solve_batch(const BatchSolveArgs& b, int j, int ps, hipStream_t s);
hipError_t launch_reduce_batch(const BatchReduceArgs& b, hipStream_t s);
int cls_variant(int na, int n_slots);

// Snapshot windows of at least this many samples are imaged by all eight
// waves of a paired-engine workgroup together; shorter ones by one wave each.
constexpr int64_t kSnapGroupWindow = 64;

// Half-frame buffer of the two-waves-per-SIMD engines: the 64 rows of one
// half of the columns (32 cells each) at a pitch of 33 complex values, so
// that 64 lanes loading their own rows stay free of bank conflicts; column 32
// is the pad that the schedule's padding slots write.
constexpr int kHalfPitch = 33;

// Launchers: return hipSuccess or the launch error.  N = grid size.
// Gridding schedule geometry of the N <= 64 engine: lanes per frame and LDS
// row pitch (complex values) that slot offsets refer to.
int grid_lanes(int N);
int grid_pitch(int N);
// Slot rows available to the N = 128, 256 residue-class engine.
int cls_table_slots();
bool image_supported(int N, int na, int n_slots);
bool pair_engine(const ImageArgs& a, int N);   // the 64 x 64 two-waves-per-SIMD engine applies
bool cls_pair_engine(const ImageArgs& a, int N);   // the 128 / 256 two-waves-per-SIMD class engine applies
bool cls_dense_engine(const ImageArgs& a, int N);  // the dense two-waves-per-SIMD class engine applies
bool cls_pair_db(const ImageArgs& a, int N);       // the class-pair engine's double-buffered form applies
// Imaging workgroups per (channel, time split) of launch_image at N = 128, 256
// (class groups); 1 below.
int cls_groups(const ImageArgs& a, int N);
// Split-precision DFT-GEMM imaging (matrix cores), N = 32 or 64 directly (its
// gridding schedule has 64 N / 32 lanes and transposed (G^T) cell offsets),
// N = 128, 256 by residue classes (the class schedule slots_c).
int dft_owners(int N);
bool dft_supported(int N, int na, int n_slots);
hipError_t launch_image_dft(int N, const ImageArgs& a, hipStream_t s);
hipError_t launch_image(int N, const ImageArgs& a, hipStream_t s);
// snapshot form (a.t_acc >= 1, a.snap set; N <= 64)
hipError_t launch_image_snap(int N, const ImageArgs& a, hipStream_t s);
hipError_t launch_grid(int N, const GridArgs& a, hipStream_t s);
// n integer-format samples (ci4 / ci8) decoded as the imaging engines decode
// them, to int16 (re, im) pairs
hipError_t launch_unpack(const uint8_t* efield, int64_t n, int fmt, int16_t* out, hipStream_t s);
hipError_t launch_image_acc(int N, const ImageAccArgs& a, hipStream_t s);
hipError_t launch_reduce(const float* partial, int splits, int64_t per_split, double scale,
                         float* image, hipStream_t s);
bool solve_supported(int na, int fmt, int n_pix = 1);
// the several-pixel solve runs as a task of the fused run (kSolveMainThreads threads)
bool solve_multi_fusable(int na, int fmt);
int solve_main_j(int na);   // antennas per thread slot of the single-pixel solve
hipError_t launch_solve(const SolveArgs& a, hipStream_t s);
// The solve of these arrays runs one wave per channel (small arrays, short
// intervals): launch_solve picks it, so a batched solve leaves them to it.
bool solve_by_wave(const SolveArgs& a);
bool band_supported(int na, int fmt);
// cooperative launch; *groups receives the number of workgroups
hipError_t launch_solve_band(const BandArgs& b, int n_cu, hipStream_t s, int* groups = nullptr);
// u_hist[n] = 1 / g_hist[n] (FP64, rounded to FP32; zero for flagged antennas), n < n_int
hipError_t launch_hist_to_u(const double2* g_hist, const uint8_t* hold, int64_t n_int, int F, int Na, float2* u_hist,
                            hipStream_t s);
hipError_t launch_update(const UpdateArgs& a, hipStream_t s);
hipError_t launch_adjoint(int N, const AdjointArgs& a, hipStream_t s);
hipError_t launch_adjoint_reduce(const double2* partial, int splits, int F, int Na,
                                 const double2* gains, double scale, double2* dL_dg,
                                 hipStream_t s);
hipError_t launch_recip(const double2* gains, const uint8_t* flag, int F, int Na, float2* u,
                        hipStream_t s);

}  // namespace epic
