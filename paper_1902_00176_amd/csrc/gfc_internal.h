// gfc_internal.h - argument blocks shared by the host plan code and the kernel files.
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>

namespace gfc {

struct f2 {
  float x, y;
};

// Spectra (T1 and T2 of the forward solve, U and W of the backward one, the planes of a
// volume) are stored tile-major: within an image (or plane) of R rows and NHP bins per row,
// bins l come in tiles of 16, and a tile holds its 16 bins of row 0, then of row 1, and so on
// (complex index tile_index(y, l, R)). The column pass, whose workgroups own one tile of
// columns, then reads and writes each tile as one contiguous block; a row pass sees a row as
// 128-byte pieces, one per tile, which cost it nothing measurable against contiguous rows.
// NHP is a multiple of 32, so every row has whole tiles; an image still takes R * NHP bins.
constexpr int kTileBins = 16;
__host__ __device__ __forceinline__ int tile_index(int y, int l, int R) {
  return ((l >> 4) * R + y) * kTileBins + (l & (kTileBins - 1));
}

// ---- row passes -----------------------------------------------------------------------
// Forward row pass: for each row y in [0, H] of the divergence L (block at the torus
// origin), T1[y, l] = L^[y, l] for l > K, and the split form T1[y, l] = (1 - w_N^l) Ex^[y, l],
// SB[y, l] = Ey^[y, l] for l <= K (T1[y, 0] = 0). L is formed in float32 from the gradient
// and two rows of L share one complex FFT; the K + 1 lowest bins of Ex and Ey are direct sums.
constexpr int kLowBins = 4;  // row frequencies l <= 4 are split inside the row pass
// A plan may split more bins, K in (kLowBins, kMaxLowBins]: the bins l in (kLowBins, K] are
// then overwritten in split form by launch_low_ext after the row pass (thin, wide images).
constexpr int kMaxLowBins = 32;
// On-device gradient edits applied to every loaded pixel before the divergence:
// threshold (Sec. 3.2.3): E kept where fl(fl(gx^2) + fl(gy^2)) >= tau2, else 0;
// GDM (eq. (26)): E scaled to |E|^(1-alpha) C^alpha, orientation kept, 0 where E = 0.
// kInLaplacian: the input is the divergence itself, L [B][H+1][W+1] (Algorithm B's input).
// kIn3D: a slice z of a volume; the divergence also takes -gz[z-1] + gz[z] (7-point).
enum { kEditNone = 0, kEditThreshold = 1, kEditGdm = 2, kInLaplacian = 3, kIn3D = 4 };
struct RowFwdArgs {
  const float* gx;
  const float* gy;
  const float* C;     // [B][H][W] edge intensity (GDM), or L [B][H+1][W+1] (kInLaplacian)
  int edit;           // kEdit*
  float tau2;         // threshold: tau^2 rounded to float32
  float alpha;        // GDM weight in [0, 1]
  f2* T1;             // [B] images of (H+1) x NHP, tile-major (NHP = NH rounded up to 32)
  f2* SB;             // [B][H][KP]     (KP = side-array row stride >= K + 1)
  const f2* twA;      // [N1][N2]: w_N^(k1 j), forward sign
  const f2* twL;      // [2][kLowBins+1][G]: (1 - w_N^l) w_N^(l j) and w_N^(l j), 0 for j >= N2
  const f2* twX;      // [N + kMaxLowBins + 1]: w_N^m (m < N), then 1 - w_N^l (l <= kMaxLowBins)
  int H, W, K, KP;
  int N, NHP;         // row length and bins per T1 row (used by launch_low_ext)
  int npairs;         // ceil((H+1) / 2)
  long long img_in, img_t1, img_sb;
  // volumes (kIn3D): the launch's image index runs over (volume, z) with z in [0, zd]; gx,
  // gy, gz are [B][zd][H][W]; T1 planes are [B][zp] of (H+1) x NHP (plane z of each volume)
  const float* gz;
  int zd, zp;
  f2* SZ;             // volumes: [B][zp][H][KP] row sums of gz for bins l <= K (plane z < zd)
};

// Inverse row pass: rows y in [0, H) of T2 (already scaled by 1/N), two rows per complex
// inverse FFT; u[y, x] = v[y, x] - v_ref for x in [0, W).
struct RowInvArgs {
  const f2* T2;       // [B][>=H][NH] with row stride NH
  float* u;           // [B][H][W]
  const double* partial;  // [B][nparts]: v_ref = sum of the partials
  int nparts;
  const f2* twB;      // [N2][N1]: w_N^(k j2), forward sign, conjugated in use
  int H, W;
  int npairs;         // ceil(H / 2)
  long long img_t2, img_u;
  double* mom;        // [B][gridDim.x][2]: sums of u and u^2 per workgroup, or null
  // volumes: the image index runs over (volume, z), z < zd; T2 planes [B][zp] of (H+1) x NHP,
  // partials [B][nparts] per volume (zd = zp = 1 for images)
  int zd, zp;
  int N;              // row length (the ragged launches covering several lengths branch on it)
};

// Bins kLowBins < l <= K of T1 and SB in the split form, as direct float32 sums over the
// (edited) gradient rows; run after the row pass on the same stream. No-op for K <= kLowBins.
hipError_t launch_low_ext(const RowFwdArgs& a, int B, hipStream_t s);
// Laplacian input, bins l <= K: the column pass takes these bins in the split form
// a + (1 - S) b. For a given L they are written as b[y, l] = P[y, l] (y < H), a[y, l] = 0 for
// y < H and a[H, l] = P[H, l], with P[y, l] = sum_{y' <= y} L^[y', l] the running sum over
// rows of the row spectra; then a + (1 - S) b = L^ row by row, and the column sums, which
// the Green's function amplifies most, are P's last row: a single value, never a difference
// of rounded ones. L^[y, l] are direct sums with float64 twiddles and accumulation, P is a
// float64 scan (fixed order); each is rounded once to float32.
struct LapLowArgs {
  const float* L;     // [B][H+1][W+1]
  const double* twD;  // [N][2]: w_N^m = (cos, -sin)(2 pi m / N), float64
  double* Lh;         // [B][H+1][K+1][2]: L^[y, l] (workspace)
  f2* T1;             // [B] images of (H+1) x NHP, tile-major
  f2* SB;             // [B][H][KP]
  int H, W, N, K, NHP, KP;
  long long img_L, img_lh, img_t1, img_sb;
};
hipError_t launch_lap_low(const LapLowArgs& a, int B, hipStream_t s);

// Colour correction of eq. (25) in place on u [B][npix]: every workgroup of image b reduces
// that image's nparts moment pairs in a fixed order, then u <- (u - mean) * I_std[b] / std + I_mean[b].
hipError_t launch_color_apply(float* u, const double* mom, int nparts, const float* I_mean,
                              const float* I_std, long long npix, int B, hipStream_t s);

// Backward row pass 1: R2C of du rows (two rows per complex FFT), U[y, l], l in [0, NH);
// also per-block partial sums of du for sum(du).
struct RowBwdFwdArgs {
  const float* du;
  f2* U;              // [B][H+1][NH]
  double* sums;       // [B][gridDim.x]
  const f2* twA;
  int H, W;
  int npairs;
  long long img_in, img_u;
};

constexpr int kLowBinsB = 64;  // Kb: backward columns l <= Kb take -D_y inside the recursion

// Backward row pass 2: per row y in [0, H): Zx = (1 - w_N^-l) Wv[y, l],
// Zy = SD[y, l] (l <= Kb) or Wv[y, l] - Wv[y+1, l] (l > Kb); one complex inverse FFT of
// Zx + i Zy gives (dgx, dgy) on row y.
struct RowBwdInvArgs {
  const f2* Wv;       // [B][H+1][NH]
  const f2* SD;       // [B][H][KbP]
  float* dgx;
  float* dgy;
  const f2* twB;
  int H, W, Kb, KbP;
  long long img_w, img_sd, img_out;
};

// ---- column pass ------------------------------------------------------------------------
// Per column frequency l the column Green's function 1/lambda(., l) is applied exactly as
// -rho (1 - rho S^-1)^-1 (1 - rho S)^-1 on Z_M (two first-order recursions, float64), with
// rho the root < 1 of rho + 1/rho = 2 + 4 sin^2(pi l / N). All constants are float64 from
// the host.
struct ColConst {
  double rho;       // recursion root (column 0: 1, handled separately)
  double inv_rho;   // 1 / rho
  double omr;       // 1 - rho (computed without cancellation)
  double outs;      // output scale: -rho / N  (column 0: 1 / N)
  double rhoL;      // rho^Lseg
  double rhoLl;     // rho^Llast
  double gL;        // (1 - rho^(2 Lseg)) / (1 - rho^2)
  double gLl;       // (1 - rho^(2 Llast)) / (1 - rho^2)
  double cg;        // gamma = cg * c[R-1] (+ cgd * dv)
  double rhoRm1;    // rho^(R-1)
  double cT;        // z[R] = cT * w[R-1] + czR * Sum_w (+ cTd * dv)
  double czR;
  double ra, rb;    // forward: z[r0] = ra * w[R-1] + rb * z[0]
  double cgd, cTd;  // backward: Dirac at r0 terms
  double wre, wim;  // forward: reference term = wre * Re(z[r0]) - wim * Im(z[r0])
  int kseg;         // segments over which rho^distance stays above 2^-64 (capped at nseg)
  int pad_;
};

// Column geometry. A column of R input rows is cut into nseg segments of Lseg rows (one
// thread each), the last one Llast rows long. When the zero rows of the torus allow it the
// block is treated as Rp = nseg * Lseg rows (the extra rows are zeros of the torus that
// read as 0 past the end of the buffer), so every segment is full; otherwise (tail) Rp = R.
// All recursion constants use Rp.
struct ColGeom {
  int C, nseg, Lseg, Llast, Rp;
  bool tail;
};

struct ColFwdArgs {
  f2* T;              // in: T1, [B] tile-major (H+1) x NHP; out (in place): T2 rows [0, H)
  const f2* SB;       // [B][H][KP]
  const ColConst* cc; // [NH]
  double* partial;    // [B][nparts]: per column-tile sums of the reference terms
  int nparts;         // column tiles
  int tile0;          // first tile of this launch (set by the launcher)
  int H, M, NH, NHP, K, KP, r0;
  int C, nseg, Lseg, Llast, Rp;   // R = H + 1 rows of input
  long long img_t, img_sb;
  // volumes: the image index runs over (volume, kz); constants cc[kz][NH]; the DC path only
  // at kz = 0 (zp = 1 for images)
  int zp;
};

struct ColBwdArgs {
  f2* T;              // in: U, [B] tile-major (H+1) x NHP, rows [0, H); out: W rows [0, H]
  f2* SD;             // out: [B][H][KbP]
  const ColConst* cc; // [NH]
  const double* sums; // [B][nsums]: sum(du) = sum of the partials
  const f2* dshift;   // [NH]: w_N^(l c0) (forward sign): row DFT of a Dirac at column c0
  int nsums;
  int H, M, NH, NHP, Kb, KbP, r0;
  int C, nseg, Lseg, Llast, Rp;   // R = H rows of input
  long long img_t, img_sd;
  int nimg;           // images of the launch (B)
  int tile0;          // first tile of this launch (set by the launcher)
};

// ---- ragged batches ---------------------------------------------------------------------
// One launch covers many images of different sizes: each workgroup takes one work item
// (image, block of that image's grid) and the image's argument block from a table built
// once on the host. Buffer addresses in the tables are offsets from the bases passed at
// launch: input/output elements, workspace bytes.
struct RgItem {
  int img, blk;
};
struct RgBase {
  const float* gx;
  const float* gy;
  float* u;
  unsigned char* ws;
};
// The ragged kernels read the bases from a device slot, written on the launch stream by
// launch_set_base just before them: a captured graph then serves any buffer addresses.
struct RgRowFwd {
  RowFwdArgs a;
  long long in, t, side;
};
struct RgCol {
  ColFwdArgs a;
  long long t, side, red;
};
struct RgRowInv {
  RowInvArgs a;
  long long out, t, red;
};

// ---- z transforms of volumes -------------------------------------------------------------
struct ZfftArgs {
  f2* T;               // spectra of one volume at T + vol * vol_stride: [P] planes of R x NHP
  const f2* tw;        // [P1][P2]: w_P^(k1 j), forward sign
  int R, NH, NHP;      // rows per plane, row frequencies used, bins per row
  int tiled;           // planes tile-major (the spectra T), else row-major (side arrays)
  int din, dout;       // planes read (the rest are zero), planes written
  long long plane, vol_stride;  // elements per plane, per volume
};
struct ZKernels {
  int P, P1, P2;
  hipError_t (*run)(const ZfftArgs&, int sign, int B, hipStream_t);
};
const ZKernels* find_z_kernels(int P);
// total[b] = sum of partial[b][0 .. nparts) in a fixed order, one workgroup per volume
hipError_t launch_partial_sums(const double* partial, int nparts, double* total, int B,
                               hipStream_t s);
// Volumes, after the z transforms of T and of the side array SZ (row sums of Ez): the split
// bins take the z difference as its symbol, T[vol][kz][y][l] += (1 - w_P^kz) SZ[vol][kz][y][l]
// for y < H, l <= K (omz[kz] = 1 - w_P^kz, float64-built).
hipError_t launch_sz_combine(f2* T, const f2* SZ, const f2* omz, int H, int NHP, int K, int KP,
                             int P, long long plane_t, long long plane_s, int B, hipStream_t s);

// launchers (defined in the kernel files)
// The split N = N1 * N2 of one row pass's four-step FFT: lane slots of G lanes, `slots` of
// them per workgroup. Each pass of a row length has its own (chosen by the autotuner).
struct RowSplit {
  int N1, N2, G, slots;
};
struct RowKernels {
  int N;
  // plain forward, other forward modes (edits, Laplacian input, volume slices), inverse,
  // backward forward and backward inverse row passes
  RowSplit f, e, i, bf, bi;
  hipError_t (*fwd)(const RowFwdArgs&, int B, hipStream_t);
  hipError_t (*inv)(const RowInvArgs&, int B, hipStream_t);
  hipError_t (*bfwd)(const RowBwdFwdArgs&, int B, hipStream_t);
  hipError_t (*binv)(const RowBwdInvArgs&, int B, hipStream_t);
  hipError_t (*rg_fwd)(const RgBase*, const RgRowFwd*, const RgItem*, int nitems, bool half,
                       hipStream_t);
  hipError_t (*rg_inv)(const RgBase*, const RgRowInv*, const RgItem*, int nitems, bool half,
                       hipStream_t);
};
const RowKernels* find_row_kernels(int N);
// the entry for N whose forward row pass uses N1 (a library built for split tuning holds one
// entry per candidate split; the default library one per length)
const RowKernels* find_row_kernels_split(int N, int N1);
// ragged launches that cover several row lengths of one workgroup size (half support only)
struct RgMulti {
  int id;  // distinct per group of lengths
  hipError_t (*fwd)(const RgBase*, const RgRowFwd*, const RgItem*, int nitems, hipStream_t);
  hipError_t (*inv)(const RgBase*, const RgRowInv*, const RgItem*, int nitems, hipStream_t);
};
const RgMulti* find_rg_multi(int N);
int row_kernel_count();
const RowKernels* row_kernel_at(int i);

hipError_t launch_col_fwd(const ColFwdArgs& a, int B, hipStream_t s, hipStream_t side = nullptr,
                          hipEvent_t fork = nullptr, hipEvent_t join = nullptr);
hipError_t launch_col_bwd(const ColBwdArgs& a, int B, hipStream_t s, hipStream_t side = nullptr,
                          hipEvent_t fork = nullptr, hipEvent_t join = nullptr);
// ragged forward column pass: items of tiles holding columns l <= K and of the others,
// one workgroup shape (threads, LDS bytes) for all images, rows per segment Lseg
hipError_t launch_col_fwd_rg(const RgBase* base, const RgCol* tab, const RgItem* low,
                             int nlow, const RgItem* rest, int nrest, int Lseg, bool tail,
                             int threads, size_t shm, hipStream_t s);
constexpr int kColMaxThreads = 1024;  // largest column-pass workgroup
// ragged low-bin extension: items (image, row y <= H) of the images whose plan has K > kLowBins
hipError_t launch_low_ext_rg(const RgBase* base, const RgRowFwd* tab, const RgItem* items,
                             int nitems, hipStream_t s);

}  // namespace gfc
