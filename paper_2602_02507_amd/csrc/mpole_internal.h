// Internal interfaces between the host plan (plan.cpp) and the gfx950 kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <cstddef>
#include <cstdint>

namespace mpole {

constexpr double kPi = 3.14159265358979323846264338327950288;
constexpr int kGaussNodes = 16;   // Gauss-Legendre points per theta sub-interval
// nAM and the block count of each class are padded to a multiple of the K
// step of the contraction kernels (16 for both the f64 and the split kernels)
constexpr int kPadF64 = 16;
constexpr int kPackSpan = 1024;   // blocks of one shell per packing workgroup
constexpr int kTsumChunks = 64;   // block chunks of the bind-time column sums of a table
constexpr int kShiftSamples = 4;  // blocks sampled per shell for its mean source density
// Blocks with more member cells than this are reduced and broadcast by one
// workgroup each (kernels that give a block to one thread skip them).
constexpr int kLargeBlock = 64;
// Members per workgroup of a large block (larger blocks are split into
// chunks whose partial sums are combined in chunk order).
constexpr int kLargeChunk = 4096;
// Rows of single cells copied per workgroup by the band kernel.
// modes per workgroup of the radial scan (x 8 bytes of each row; namp is a
// multiple of 16): 16 when that still gives a workgroup per CU, else 8 (twice
// the workgroups, shorter row segments); every field of a batch takes 8
constexpr int kScanModesWide = 16, kScanModesNarrow = 8, kScanWideMinWgs = 256;
// BF16 x3 separable: one-row blocks of up to this many phi cells are averaged
// inside the phi transforms (a power of two, at most 8)
constexpr int kSepFuseNk = 8;
// single-cell rows merged into one theta band (at most), and single-cell
// rows (with their mirror rows) per packing workgroup of a banded class
constexpr int kBandRows = 8;
constexpr int kBandCopyRows = 4;
// FP16 x2: pairs of one shell's row split into planes per workgroup
constexpr int kSplitRowChunk = 1024;
// bands of merged blocks copied per group of loads in the broadcast phase
constexpr int kBcastBands = 4;

// Gauss-Legendre rule on [-1, 1], computed on the host.
struct GaussRule {
  double x[kGaussNodes];
  double w[kGaussNodes];
};

// Per-coarsening-class device view (lives in the workspace).
struct ClassDev {
  const int32_t *rows;   // [nrows] global shell of each class row, ascending
  const int32_t *moff;   // [nblocks+1] CSR offsets of block members
  const int32_t *mem;    // [ncell] member fine-cell index j*nphi+k, ascending per block
  const int4 *rect;      // [nblocks] (j0, k0, nj, nk) when every block is a theta-phi rectangle, else null
  const int32_t *span0;  // [ceil(nblocks / kPackSpan)] first cell of a span of consecutive single-cell blocks, else -1
  const int32_t *pspan0; // [ceil(npair / kPackSpan)] first rep cell of a packing span of pairs whose rep blocks
                         // are single cells at consecutive cells (their mirrors then are the mirror cells), else -1
  const int32_t *lidx;   // [nblocks] index of a large block in the class's large-block list, else -1; null if none
  // theta bands when every block is an nj x nk rectangle at a phi column
  // that is a multiple of nk, uniform within the band: (j0, nj, nk, kind),
  // kind 0 = single cells (up to kBandRows rows), 1 = blocks of at most
  // kLargeBlock cells with nk a power of two <= 64, 2 = larger blocks; null
  // for other block maps
  const int4 *bands;
  int32_t nbands;
  // indices of the bands of merged blocks (kind 1): the expansion writes the
  // first cell of each such block, the broadcast phase the rest
  const int32_t *bcast;
  int32_t nbcast;
  // The contractions run over block pairs.  With the mirror fold (PlanDev::
  // fold) a pair is a block and its mirror image about the equator (theta ->
  // pi - theta), whose kernels differ only by the sign (-1)^(l+m); a block
  // that is its own mirror, and every block of an unfolded plan, is a pair
  // (b, b).  Pairs are ordered by their first block.
  const int2 *pairs;     // [npair] (rep, mir) block ids
  int32_t npair, npair_pad;
  // packing: band tasks (j0, nj, nk, q0), one workgroup each (null: spans of
  // kPackSpan pairs), and the packing workgroups per shell of this class
  const int4 *ptasks;
  int32_t npack;
  double *table;         // [nblocks_pad][namp] FP64 block-mean kernels, natural mode order, zero padded
  double *tm, *te;       // FP64 contraction operands over pairs: [npair_pad][namp_m] (moment) and
                         // [npair_pad][namp_e] (expansion); both the table itself when unfolded
  double *tcol0;         // [npair_pad] l = 0 kernel of each pair (contiguous)
  uint16_t *tplanes;     // [nplanes] split planes of te, rows = pairs, k = expansion mode column
  uint16_t *ttplanes;    // [nplanes] split planes of tm transposed, rows = moment mode column, k = pairs
  // packed sources over pairs: even = S(rep) + S(mir), odd = S(rep) - S(mir)
  // (the mirror's own source is left out of a pair (b, b)); odd only folded
  double *pack, *pack_o;        // [nrows][npair_pad] FP64 (FP64 and FP16 x2 paths)
  uint16_t *ppacks, *ppacks_o;  // [nplanes] split planes, rows = class rows, k = pairs, row-major
                                //   [row][k/16][plane][k%16] (each shell's row contiguous)
  double *pscale;        // [nrows] power-of-two row scales of the packed source
  double *partial;       // [splits][nrows][namp_m] split-K partial moments (moment mode columns)
  double *wsum;          // [nblocks_pad] 4 pi G dOmega of each block (sum over its cells)
  double *tsum;          // [namp] sum_b wsum[b] table[b][n], summed over b in order
  int32_t nrows, nblocks, nblocks_pad;
  int32_t splits, kchunk;             // moment split-K over pairs: splits x kchunk >= npair_pad
  int32_t m_tiles_mom, m_tiles_exp, n_tiles_mom, n_tiles_exp;   // tiles of the contractions
  int32_t wg_mom_begin, wg_exp_begin;  // prefix sums over classes
};

// Whole-plan device view.
struct PlanDev {
  int32_t nr, ntheta, nphi, lmax, nam, namp, ncell, nclasses, nplanes;
  double G;
  const double *r_edges, *theta_edges, *phi_edges;  // device copies
  const int32_t *shell_class;  // [nr]
  const int32_t *shell_row;    // [nr] row of each shell within its class
  ClassDev *classes;           // [nclasses] (device copy)
  double *pavg;      // [ntheta][nplm] theta-cell averages of P~_l^m
  double *trig;      // [nphi][2*(lmax+1)] (<cos m ph>, <sin m ph>)
  double *weight;    // [ncell] 4 pi G dOmega = wrow[j] * dphi[k]
  double *wrow;      // [ntheta] 4 pi G (cos th_j - cos th_j+1)
  double *dphi;      // [nphi] phi_k+1 - phi_k
  double *dom;       // [ncell] dOmega, the solid angle of each angular cell
  double *jr, *ji;   // [nr][lmax+1] exact shell integrals of r^(2+l), r^(1-l)
  double *rr, *ri;   // [nr][lmax+1] volume-averaged r^l, r^-(l+1)
  double *ang;       // [nr][namp] reduced angular moments
  double *coef;      // [nr][namp] expansion coefficients
  // Mode columns of the contractions.  Folded: the moment N dimension holds
  // the even modes (l + m even) padded to odd_m0 (a multiple of the tile
  // width, so that every output tile has one parity), then the odd modes,
  // namp_m columns in all; the expansion K dimension holds the even modes
  // padded to odd_e0 (a multiple of 16), then the odd modes, namp_e in all.
  // Unfolded: natural order, namp_m = namp_e = odd_m0 = odd_e0 = namp, null maps.
  int32_t fold;
  int32_t namp_m, odd_m0, namp_e, odd_e0;
  const int32_t *pos_m;    // [namp] natural mode -> moment column, -1 past nam (null: identity)
  const int32_t *perm_m;   // [namp_m] moment column -> natural mode or -1 (null: identity)
  const int32_t *perm_e;   // [namp_e] expansion column -> natural mode or -1 (null: identity)
  double *coef_e;    // [nr][namp_e] coefficients in expansion columns (FP64 folded), else coef
  uint16_t *cplanes; // [nplanes] split planes of coef, rows = shells, k = expansion column
  double *cscale;    // [nr] row scales of coef
  double *mono_part; // [nr][mono_stride] FP64 partial monopole moments (split precisions), or null
  double *max_part;  // [nr][mono_stride] partial row maxima of the packed source (FP16 x2)
  int32_t mono_stride;
  int32_t pack_parts;       // packing workgroups per shell
  int32_t split_chunks;     // FP16 x2: row-split workgroups per shell (kSplitRowChunk pairs each), else 0
  const int2 *bcast_items;  // broadcast workgroups: (shell, first band), kBcastBands bands each
  int32_t wg_mom, wg_exp;   // workgroups of the two contraction launches
  int32_t tm_mom, tm_exp;   // output tile heights of the two contractions
  double *edge_r, *edge_i;  // [nr+1][namp] edge moments when the caller passes no buffer
  double *shift;            // [nr] per-shell mean source density removed before splitting (split precisions)
  double *tsum_part;        // [kTsumChunks][namp] bind-time partial sums of tsum
  // blocks with more than kLargeBlock members, over all shells: items
  // (shell, block) in shell order, the first item of each shell, and the
  // block sources sum 4 pi G dOmega rho of the dense paths; each item is
  // split into chunks of at most kLargeChunk members: (item, chunk of the
  // item, chunks of the item, first chunk of the item) and their partial
  // (weighted sum, weight) pairs
  const int2 *litems;       // [n_litems]
  const int32_t *lbase;     // [nr + 1]
  double *lsum;             // [n_litems] (dense paths), or null
  const int4 *lchunks;      // [n_lchunks]
  double *lpart;            // [n_lchunks][2]
  int32_t n_litems, n_lchunks;
  int32_t max_bands;        // most bands of any class
};

// Phases of one solve; a launch of phase h covers the workgroups
// [prefix[h][f], prefix[h][f+1]) of every field f of a batch.
enum Phase { PH_PACK = 0, PH_SPLITROWS, PH_MOMENT, PH_REDUCE, PH_SCAN, PH_COEF, PH_EXPAND, PH_BCAST, PH_COUNT };

// Per-field device pointers of one solve.
struct SolveIO {
  const double *rho;
  double *phi, *ang, *interior, *exterior;
};

// What a solve-time kernel gets: one or more fields (plans) and their I/O.
struct BatchDev {
  const PlanDev *plans;        // [nf] device copies
  const SolveIO *io;           // [nf] device array, or null: use io1 (single plan)
  SolveIO io1;
  const int32_t *prefix;       // [PH_COUNT][nf+1] workgroup prefix sums
  int32_t nf;
  unsigned long long *stamps;  // [nf+1]: per field, wall clock when its potential is done; [nf] batch start; or null
};

// Work queues of the persistent batched solve (device copies in the batch
// workspace): one queue per XCD, a run of segments (field, phase, first
// item, items) with ascending first items.  Phase h of field f has
// sub[f][h] per-phase workgroups (sub-items), run grp[f][h] at a time as one
// item.  Dispensers per queue, completion counters and items per (field,
// phase), the error word.
struct PersistDev {
  const int4 *segs;      // all queues' segments, queue after queue
  const int32_t *qseg;   // [nq + 1] segment range of each queue
  const int32_t *xcc_q;  // [16] queue of each XCD id, -1 for none
  const int32_t *sub;    // [nf][PH_COUNT] sub-items of each phase
  const int32_t *grp;    // [nf][PH_COUNT] sub-items per item
  int32_t nq;
  uint32_t *next;        // [nq] next item of each queue
  uint32_t *done;        // [nf][PH_COUNT] completed items
  const int32_t *tot;    // [nf][PH_COUNT] items of each phase
  uint32_t *err;         // 1: a dependency wait ran out of polls
};

// Separable FP64 path: bind-time transform tables and per-solve intermediates
// (trig modes t = 0, 2m-1 (cos), 2m (sin), padded to tpad; t-major per shell).
struct SepClass;
struct SepDev {
  int32_t tpad;
  int32_t max_src, max_avg;   // longest per-class block lists below
  double *tw;              // [2][tpad][nphi]: dphi_k <trig_t>_k, then <trig_t>_k
  double *pw;              // [L+1][ntheta][L+1]: 4 pi G dcos_j <P~_{l'+m,m}>_j as [m][j][l']
  double *pt;              // [L+1][L+1][ntheta]: <P~_{l'+m,m}>_j as [m][l'][j]
  double *shat;            // [nr][ntheta][nphi] block-mean density on rows with a merged block
  const uint8_t *rowalt;   // [nr][ntheta] 1 where the row reads shat
  double *f, *g;           // [nr][tpad][ntheta] phi analysis, theta synthesis
  const double *dom;       // [ntheta][nphi] solid angle of each cell (the plan's table)
  const SepClass *cls;     // [nclasses] per-class block lists (device copy)
  // BF16 x3 phi transforms (null for FP64): the m >= 1 rows of TW and TT
  // split into bf16 planes and stored in MFMA fragment order, 64 lanes x 16
  // bytes per (32-deep K step, 16-row tile, plane):
  //   twf [ks_a][mt_a][3][64]: lane l holds TW[1 + 16 mt + l % 16][32 ks + 8 (l / 16) + e], e < 8
  //   ttf [ks_s][nt_s][3][64]: lane l holds TT[1 + 32 ks + 8 (l / 16) + e][16 nt + l % 16]
  // (zero past t = 2L or k = nphi)
  const uint32_t *twf, *ttf;
  int32_t ks_a, mt_a, ks_s, nt_s;
  // BF16 x3: rows whose blocks are one row of at most fuse_nk (<= 8) cells
  // are averaged inside the phi transforms (rowalt = 1 + log2 nk there, 1 for
  // rows read from shat); 0: none
  int32_t fuse_nk;
};
// Per class: blocks on rows with a merged block (source means), and blocks
// with more than one member (potential means); device lists, without the
// blocks of more than kLargeBlock members (those go through launch_large).
struct SepClass {
  const int32_t *src;
  int32_t n_src;
  const int32_t *avg;
  int32_t n_avg;
};

// Thread-local error message of the C ABI: fail() sets it and returns code,
// ok() clears it and returns MPOLE_OK (defined in plan.cpp).
int fail(int code, const char *fmt, ...) __attribute__((format(printf, 2, 3)));
int ok();

// Split precisions: operands are sums of nplanes narrow floats (hi + mid + lo),
// stored as raw 16-bit patterns.
enum SplitKind { kSplitBf16x3 = 1, kSplitFp16x2 = 2 };

// ---- launchers (all asynchronous on `s`; return hipSuccess or the launch error)
// bind time, per plan
hipError_t launch_fill_zero(void *p, size_t bytes, hipStream_t s);
hipError_t launch_fill_word(void *p, size_t bytes, uint32_t word, hipStream_t s);   // every 32-bit word = word
hipError_t launch_fill_value(double *p, size_t n, double v, hipStream_t s);
hipError_t launch_tables(const PlanDev &P, const ClassDev *host_classes, const GaussRule &g, bool dense,
                         hipStream_t s);
hipError_t launch_split_tables(const PlanDev &P, const ClassDev *host_classes, int kind, hipStream_t s);
// per-pair tables of the dense paths: the l = 0 kernel of each pair, and for
// the folded FP64 path the operands tm and te (after launch_tables)
hipError_t launch_pair_tables(const PlanDev &P, const ClassDev *host_classes, hipStream_t s);
// solve time, one launch per phase covering every field of B; wgs = total workgroups
// (prefix[h][nf]); precision = the fields' common precision (0 = FP64)
hipError_t launch_stamp_reset(const BatchDev &B, hipStream_t s);
hipError_t launch_stamp(unsigned long long *stamps, int idx, hipStream_t s);   // stamps[idx] = wall clock
hipError_t launch_pack(const BatchDev &B, int precision, int wgs, hipStream_t s);
hipError_t launch_split_rows(const BatchDev &B, int wgs, hipStream_t s);   // FP16 x2 only
// every cell of the merged blocks of banded classes from the block's first cell
hipError_t launch_bcast(const BatchDev &B, int wgs, hipStream_t s);
hipError_t launch_moment(const BatchDev &B, int precision, int wgs, hipStream_t s);
hipError_t launch_reduce(const BatchDev &B, int wgs, hipStream_t s);
hipError_t launch_scan(const BatchDev &B, int wgs, int modes, hipStream_t s);
hipError_t launch_split_coef(const BatchDev &B, int precision, int wgs, hipStream_t s);
hipError_t launch_expand(const BatchDev &B, int precision, int wgs, hipStream_t s);
hipError_t launch_gradient(const PlanDev &P, const double *phi, double *d_r, double *d_th, double *d_ph, int periodic,
                           hipStream_t s);
// out[0..2] = -rho dPhi/dx^i, out[3] = -rho sum_i v^i dPhi/dx^i (any pointer may be null)
hipError_t launch_gravity_sources(const PlanDev &P, const double *phi, const double *rho, const double *const v[3],
                                  double *const out[4], int periodic, hipStream_t s);
// block volume average of a cell field (host copies of the class views give the spans per class);
// blocks of more than kLargeBlock members are left to launch_large
hipError_t launch_coarsen(const PlanDev &P, const ClassDev *host_classes, const double *in, double *out,
                          hipStream_t s);
// one workgroup per large block of every shell (P.litems):
//   kLargeMean   out = solid-angle weighted block mean of in, on every member (in == out allowed)
//   kLargeSum    P.lsum[item] = sum over members of P.weight * in
//   kLargeBcast  out on every member = out at the block's first member
enum LargeMode { kLargeMean = 0, kLargeSum = 1, kLargeBcast = 2 };
hipError_t launch_large(const PlanDev &P, int mode, const double *in, double *out, hipStream_t s);
// the classes with theta bands: kBandCoarsen writes the block mean of in
// (solid-angle weights) to every cell of out, copying single cells;
// kBandMean only does the bands of merged blocks of at most kLargeBlock
// cells (in == out allowed)
enum BandMode { kBandCoarsen = 0, kBandMean = 1 };
// skip_nk > 0 leaves out the bands of one-row blocks of at most skip_nk
// cells (the BF16 x3 separable path averages those inside its phi transforms)
hipError_t launch_bands(const PlanDev &P, int mode, const double *in, double *out, hipStream_t s, int skip_nk = 0);

// separable FP64 path (single plan)
hipError_t launch_sep_tables(const PlanDev &P, const SepDev &S, hipStream_t s);
hipError_t launch_sep_source(const PlanDev &P, const SepDev &S, const double *rho, hipStream_t s);
hipError_t launch_sep_phi_anal(const PlanDev &P, const SepDev &S, const double *rho, hipStream_t s);
hipError_t launch_sep_theta_anal(const PlanDev &P, const SepDev &S, double *ang_out, hipStream_t s);
hipError_t launch_sep_theta_syn(const PlanDev &P, const SepDev &S, hipStream_t s);
hipError_t launch_sep_phi_syn(const PlanDev &P, const SepDev &S, double *phi, hipStream_t s);
// BF16 x3 phi transforms of the separable path (S.twf, S.ttf set)
hipError_t launch_sep_split_tables(const PlanDev &P, const SepDev &S, hipStream_t s);
hipError_t launch_sep_phi_anal_bf16(const PlanDev &P, const SepDev &S, const double *rho, hipStream_t s);
hipError_t launch_sep_phi_syn_bf16(const PlanDev &P, const SepDev &S, double *phi, hipStream_t s);
// the block means of the potential after a phi synthesis (merged blocks, bands, large blocks)
hipError_t launch_sep_block_means(const PlanDev &P, const SepDev &S, double *phi, hipStream_t s);

// persistent batched solve: XCD probe (ids[w] = XCD id of workgroup w),
// resident workgroups per CU of the persistent kernel of a precision (0 if
// unknown), scan modes per item, and the launch (reset + the persistent kernel)
hipError_t launch_xcc_probe(int32_t *ids, int wgs, hipStream_t s);
int persistent_blocks_per_cu(int precision);
int persistent_scan_modes();
// (Q: host copy of the descriptor, for the reset; Qdev: its device copy)
hipError_t launch_persistent(const BatchDev &B, const PersistDev &Q, const PersistDev *Qdev, uint32_t spin_limit,
                             int precision, int grid, hipStream_t s);

hipError_t launch_moment_f64(const BatchDev &B, int wgs, hipStream_t s);
hipError_t launch_expand_f64(const BatchDev &B, int wgs, hipStream_t s);


}  // namespace mpole
