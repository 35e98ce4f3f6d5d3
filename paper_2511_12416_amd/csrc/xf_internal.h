// Internal definitions shared by the host plan code (xf_host.cpp) and the
// gfx950 kernels (k_*.hip).  Not part of the public ABI.
#pragma once

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>
#include <hip/hip_vector_types.h>

namespace xf {

// Threads per workgroup of the per-bitstring kernels (four wave64s).
constexpr int kThreads = 256;
// Slots of the per-bitstring LDS hash of flip patterns.  The table is
// evaluated and cleared whenever one more batch of kThreads samples could push
// it past three quarters full, so insertion always terminates.
constexpr int kHashSlots = 2048;
// Chunk of the shared exact-mode term list evaluated per LDS pass.
constexpr int kExactChunk = 2048;
// Largest workspace region (entries) of one bitstring in the determinant-lemma
// paths.
constexpr uint64_t kEntryCapMax = 8192;
// Bytes of the fixed device scratch of xf_probabilities_noalloc (per device).
constexpr size_t kNoAllocScratchBytes = 256ull << 20;
// Empty-slot marker; valid keys use at most 63 bits.
constexpr uint64_t kEmptyKey = ~0ull;

// Snapshot of a plan's device state, passed by value to the kernels.
//
// Mode matrices (complex, (re, im) interleaved, row-major):
//   Phi0 = R_0[:, C]                                  n x m (row stride G)
//   P    = R'_L ... R'_1 Phi0                         n x m (row stride G)
//   L = 1: A1 = R'_1                                   n x n
//   L = 2: A1 = R'_2 R'_1, A2 = R'_2, R1 = R'_1        n x n,  Q = R'_1 Phi0 (n x m, stride G)
// where R'_l = R_l D0_{l-1} absorbs the d_0 phases of the CPhase layer that
// precedes rotation l.  The submatrix of trajectory x for a bitstring with
// occupied rows R is then (Sec. IV-B Eq. 16-19, extended to two layers)
//   L = 1: M = P[R,:] - 2 A1[R,N0] Phi0[N0,:]
//   L = 2: M = P[R,:] - 2 sum_{c in N0} alpha_c Phi0[c,:] - 2 A2[R,N1] Q[N1,:],
//          alpha_c = A1[R,c] - 2 A2[R,N1] R1[N1,c]
// with N_l the modes flipped an odd number of times by the d_1 choices of
// CPhase layer l.
struct DevPlan {
    int n, m, L, k, G;
    // Key of a trajectory: kind 0 = bit-compressed flip pattern (bits
    // [0, off1) are layer-0 active modes, [off1, keybits) layer-1 active
    // modes); kind 1 = the trajectory x itself (bit j <=> x_j = 1).
    int keykind, keybits, off1;
    const double2 *P, *Phi0, *A1, *A2, *Q, *R1;
    const float2 *fPhi0, *fA1, *fA2, *fQ, *fR1;
    const uint8_t *keymode;   // [64] compressed key bit -> mode
    const uint32_t *T;        // [k][k] sampling table
    const uint64_t *gkey;     // [k] key contribution of gate j
    const uint64_t *gmode;    // [k][2] mode mask of gate j's pair
    const int32_t *glayer;    // [k]
    const uint8_t *gneg;      // [k] theta_j < 0
    double scale;             // Raw Estimate: sqrt(xi*) / t
    double mixed_cond;        // XF_MIXED: largest kappa_1 of a base whose lemma products run in FP32
};

// Plan data of the general determinant-lemma evaluation (lemma_gen.h): the
// modes split into nblk blocks over which every rotation layer is
// block-diagonal, and per block its share of the input (mb columns), its
// modes touched by CPhase layer 0 (kb0 of them) and layer 1 (kb - kb0).
struct GenPlan {
    int nblk;                   // 1 or 2
    int mb[2];                  // input modes (= base rows) of each block
    int kb0[2], kb[2];          // active modes of layer 0 / of both layers per block
    int hoff[2], hsize;         // offset of each block's H in the H region; its size (complex entries)
    int hld[2];                 // row stride of each block's H (odd)
    int r1off[2], r1size;       // two layers: offset of each block's R'_1[act1, act0]; total size
    uint64_t bmask[2][2];       // modes of each block (128-bit masks)
    const uint8_t *col;         // [2][32]: input-column indices (into C) of each block
    const uint8_t *act;         // [2][64]: active modes of each block, layer 0 then layer 1
    const int8_t *pos0, *pos1;  // [128]: position of a mode in its block's active list (layer 0 / 1), or -1
    const int8_t *blk;          // [128]: block of each mode
    const uint16_t *kbt;        // [64][2]: (block << 8 | position) of the modes a key bit flips, or 0xFFFF
    const uint16_t *gpos;       // [64][2]: the same for the two modes of gate j
    // More than two CPhase layers (multi = 1): positions are (layer, mode)
    // pairs ordered by layer; with V(x) = R'_L W_{L-1} ... W_0 R'_0,
    // GA[b][r][q] = (R'_L ... R'_{l+1})[r, a], HC[b][q][c] = (R'_l ... R'_0)[a, C[c]]
    // (row stride G) and TT[b][q][q'] = (R'_l ... R'_{l'+1})[a, a'] for l > l'
    // (zero otherwise), for q = (l, a), q' = (l', a'); kb0 = kb.
    int multi;
    const double2 *GA, *HC, *TT;
};

// Exact mode: the term list as a prefix tree over the flipped positions,
// shared by every bitstring (lemma_tree.h).  An anchor is a prefix of four
// more positions than its parent's; its matrix is the Schur complement that
// eliminating them leaves on the positions its descendants still need (R).
// Anchors are stored in depth-first order, each with its own patterns.
struct TreeAnchor {
    uint32_t pat0, npat;   // its patterns: pat[pat0 .. pat0 + npat)
    uint32_t roff;         // R as indices into the parent's R: ridx[roff .. roff + nr)
    uint8_t level;         // 4 level positions eliminated (1, 2, ...)
    uint8_t nr, pnr;       // |R| and the parent's |R|
    uint8_t j[4];          // the four positions, as indices into the parent's R
    uint8_t pad;
};
struct TreePat {
    double2 w;             // summed weight of the terms with this flip pattern
    uint8_t r;             // positions beyond its anchor (0..4)
    uint8_t idx[4];        // their indices into the anchor's R
    uint8_t level;         // its anchor's level (0: the root)
    uint8_t pad[10];
};
constexpr int kTreeMaxM = 32;     // positions of the tree (all blocks)
constexpr int kTreeLevels = 8;    // anchor levels 0 (the root, all positions) .. 7
constexpr int kTreeStage = 32;    // patterns staged for one batched evaluation
struct DevTree {
    const TreeAnchor *anc;
    const uint8_t *ridx;
    const TreePat *pat;
    const uint16_t *rpos;  // [M]: (block << 8 | position) of each tree position
    const uint32_t *pstart;  // [nparts + 1]: first anchor of each part (runs of the depth-first order)
    const uint32_t *pchain;  // [nparts][8]: the ancestors of each part's first anchor, by level (1 ..)
    int nanc, nroot, npat, M, nparts;
    int slot[kTreeLevels];  // LDS offset (complex entries) of each level's matrix; slot[0]: M x M
    int toff, doff, maxr;   // LDS offsets of T (4 x maxr) and of the levels' prefix determinants
    int soff;               // LDS offset of the staged patterns (kTreeStage 4 x 4 blocks, then their factors)
    int lds;                // bytes
    double growth2;         // largest |entry|^2 / max |G|^2 accepted
};

// Per-bitstring record of the general lemma's setup kernel (see lemma_gen.h).
struct GenRec {
    double2 det;          // product over blocks of det M_B
    uint64_t shift[2];    // base pattern of each block (positions)
    uint32_t count;       // Raw Estimate: the entry count of a bitstring left to the second pattern pass
    uint32_t status;      // Raw Estimate: kRecOk, kRecZero, kRecRetry or kRecDeferred
    uint32_t pad[2];
};
// Raw Estimate setup outcomes (the setup needs only the bitstrings and
// leaves the sampler's entry counts alone; the pattern pass reads both): H
// and det ready; p = 0 written (wrong block counts or an invalid bitstring);
// base left to the workgroup setup; no acceptable base (the LU kernel takes
// the bitstring).
constexpr uint32_t kRecOk = 0, kRecZero = 1, kRecRetry = 2, kRecDeferred = 3;

// One partial gradient (of a workgroup of the lemma backward, or of a lane
// group of the LU backward; complex entries, offsets in double2):
//   oP   Gbar_P    n x G (row stride G)
//   oPhi Gbar_Phi0 n x G (row stride G)
//   oA1  Gbar_A1   n x n
//   oW   exact-mode angle-weight sums, k entries
//   oG   .x = sum of g_b over the bitstrings that contributed
struct GradLayout {
    int stride, oP, oPhi, oA1, oW, oG;
};

// Launchers (k_*.hip).  Return hipSuccess or the launch error.
hipError_t launch_zero_u64(unsigned long long *p, hipStream_t s);
// The fused Raw Estimate kernel (LU per distinct pattern) over the bitstrings
// [b0, b0 + nb) (with only != NULL: those with only[i] == kEntryDeferred) on
// `grid` workgroups (grid <= 0: one per bitstring, at most 2^20); the
// determinant-lemma paths are launch_lemma_chunk and launch_gen_chunk.
// raw_estimate_uses_lemma: the eta <= 16 one-layer lemma kernels apply
// (algorithm 0 automatic, 1 LU).
hipError_t launch_raw_estimate(const DevPlan &p, bool mixed, const uint64_t *bits, int64_t b0, int64_t nb, int64_t t,
                               uint64_t seed, double *prob, double *amp, double *logp, unsigned long long *nterm,
                               const uint32_t *only, int grid, hipStream_t s);
bool raw_estimate_uses_lemma(const DevPlan &p, int algorithm);
// Determinant-lemma Raw Estimate for bitstrings [b0, b0 + nb): the sampler
// kernel writes each bitstring's distinct (pattern, count) entries to its
// region of ekey / ecnt (cap entries each, count in ecount[i]); ev_mid
// (nullable) is recorded between it and the evaluation kernel.
uint64_t lemma_entry_cap(int64_t t);
hipError_t launch_lemma_chunk(const DevPlan &p, const uint64_t *bits, int64_t b0, int64_t nb, int64_t t,
                              uint64_t seed, uint64_t *ekey, int2 *ecnt, uint32_t *ecount, uint64_t cap,
                              double *prob, double *amp, double *logp, unsigned long long *nterm,
                              hipEvent_t ev_mid, hipStream_t s);
// Determinant-lemma backward for bitstrings [b0, b0 + nb): the sampler kernel
// refills the workspace (with resample false the workspace already holds the
// forward call's patterns of these bitstrings), then k_bwd_entries adds each
// bitstring's adjoint into
// workgroup partial i of part (nparts of them, stride lay.stride); bitstrings
// it cannot take get ecount = kEntryDeferred (see launch_raw_estimate_bwd).
bool backward_uses_lemma(const DevPlan &p, int algorithm);
size_t bwd_lemma_lds(const DevPlan &p);
hipError_t launch_lemma_bwd_chunk(const DevPlan &p, const uint64_t *bits, int64_t b0, int64_t nb, int64_t t,
                                  uint64_t seed, uint64_t *ekey, int2 *ecnt, uint32_t *ecount, uint64_t cap,
                                  const double *g, double2 *part, int nparts, const GradLayout &lay,
                                  bool resample, hipStream_t s);
// Exact mode with the LU per term over bitstrings [0, B) (only: those with
// only[b] == kEntryDeferred); grid <= 0: one workgroup per bitstring.
hipError_t launch_exact(const DevPlan &p, bool mixed, const uint64_t *keys, const double2 *w, int64_t nkeys,
                        const uint64_t *bits, int64_t B, double *prob, double *amp, double *logp,
                        unsigned long long *nterm, const uint32_t *only, int grid, hipStream_t s);
// LU backward kernels: every lane group (kThreads / G per workgroup) adds into
// its own partial, so nwg workgroups use nwg * kThreads / G partials.  With
// only != NULL just the bitstrings i of [b0, b0 + nb) with only[i] ==
// kEntryDeferred are taken.
hipError_t launch_raw_estimate_bwd(const DevPlan &p, bool mixed, const uint64_t *bits, int64_t b0, int64_t nb,
                                   int64_t t, uint64_t seed, const double *g, double2 *part, int nwg,
                                   const GradLayout &lay, const uint32_t *only, hipStream_t s);
hipError_t launch_exact_bwd(const DevPlan &p, bool mixed, const uint64_t *keys, const double2 *w,
                            const double2 *dw, int64_t nkeys, const uint64_t *bits, int64_t B,
                            const double *g, double2 *part, int nparts, const GradLayout &lay,
                            hipStream_t s);
hipError_t launch_fill_zero(double *p, size_t count, hipStream_t s);
hipError_t launch_fill_u32(uint32_t *p, int64_t count, uint32_t v, hipStream_t s);
hipError_t launch_reduce_parts(double2 *part, int nparts, int stride, double2 *out, hipStream_t s);   // overwrites part
// Raises the dynamic-LDS limit of every kernel instantiated for lane-group
// size G (k_misc.hip calls the per-file functions).
hipError_t prepare_kernels(int G);
hipError_t prepare_fused_small(int G);
hipError_t prepare_fused_g32(int G);
hipError_t prepare_fused_g64(int G);
hipError_t prepare_fused_g64x(int G);
hipError_t prepare_lemma(int G);
hipError_t prepare_bwd(int G);
// Fused LU kernels per lane-group size (k_fused_small.hip: G = 4, 8, 16;
// k_fused_g32.hip, k_fused_g64.hip); hipErrorInvalidValue for other G.
hipError_t fused_raw_small(const DevPlan &p, bool mixed, const uint64_t *bits, int64_t b0, int64_t nb, int64_t t,
                           uint64_t seed, double *prob, double *amp, double *logp, unsigned long long *nterm,
                           const uint32_t *only, int grid, hipStream_t s);
hipError_t fused_raw_g32(const DevPlan &p, bool mixed, const uint64_t *bits, int64_t b0, int64_t nb, int64_t t,
                         uint64_t seed, double *prob, double *amp, double *logp, unsigned long long *nterm,
                         const uint32_t *only, int grid, hipStream_t s);
hipError_t fused_raw_g64(const DevPlan &p, bool mixed, const uint64_t *bits, int64_t b0, int64_t nb, int64_t t,
                         uint64_t seed, double *prob, double *amp, double *logp, unsigned long long *nterm,
                         const uint32_t *only, int grid, hipStream_t s);
hipError_t fused_exact_small(const DevPlan &p, bool mixed, const uint64_t *keys, const double2 *w, int64_t nkeys,
                             const uint64_t *bits, int64_t B, double *prob, double *amp, double *logp,
                             unsigned long long *nterm, const uint32_t *only, int grid, hipStream_t s);
hipError_t fused_exact_g32(const DevPlan &p, bool mixed, const uint64_t *keys, const double2 *w, int64_t nkeys,
                           const uint64_t *bits, int64_t B, double *prob, double *amp, double *logp,
                           unsigned long long *nterm, const uint32_t *only, int grid, hipStream_t s);
hipError_t fused_exact_g64(const DevPlan &p, bool mixed, const uint64_t *keys, const double2 *w, int64_t nkeys,
                           const uint64_t *bits, int64_t B, double *prob, double *amp, double *logp,
                           unsigned long long *nterm, const uint32_t *only, int grid, hipStream_t s);
// General determinant-lemma evaluation (k_lemma_gen.hip).  gen_applies: the
// plan's sizes fit its LDS layout.  launch_gen_chunk: Raw Estimate for
// bitstrings [b0, b0 + nb) (sampler kernel into the workspace, evaluation,
// then the LU kernel for the bitstrings it deferred; with all_lu, the LU
// kernel for every bitstring).  launch_gen_exact: exact mode over [0, B) with
// flags[B] marking deferred bitstrings, then the LU kernel for those (all of
// them with all_lu); with a prefix tree (tree != nullptr), its kernel takes
// (each walk split into parts) the bitstrings whose bases need no shift
// before the pattern pass takes the rest.
bool gen_applies(const DevPlan &p, const GenPlan &g);
// gen_setup_bytes: bytes per bitstring of the setup workspace the launchers
// take in `setup` (each bitstring's H, then its base determinant and patterns).
size_t gen_setup_bytes(const GenPlan &g);
// Exact mode: segments of each bitstring's term list (a batch of fewer than
// 1024 bitstrings is spread over about 4096 workgroups); the setup workspace
// then also holds B * segments partial sums of 64 bytes after the records.
int gen_exact_segments(int64_t B, int64_t nkeys);
// Segments of the pattern pass (and of the LU kernel) after the prefix-tree
// kernel, which leaves few bitstrings: each of their term lists is split so
// that no single workgroup walks a long list.  gen_exact_part_segments: the
// segments or parts the setup workspace holds partial sums for (the largest).
int gen_tree_left_segments(int64_t nkeys);
// Parts of each bitstring's walk along the prefix tree: about kTreeWaves
// waves per call, at most one per 256 terms (and at most the plan's parts).
constexpr int kTreeWaves = 16384;
int gen_tree_parts(int64_t B, int64_t nkeys);
int gen_exact_part_segments(int64_t B, int64_t nkeys, bool tree);
hipError_t launch_gen_chunk(const DevPlan &p, const GenPlan &g, bool mixed, bool all_lu, const uint64_t *bits,
                            int64_t b0, int64_t nb, int64_t t, uint64_t seed, uint64_t *ekey, int2 *ecnt,
                            uint32_t *ecount, uint64_t cap, void *setup, double *prob, double *amp, double *logp,
                            unsigned long long *nterm, hipEvent_t ev_mid, hipStream_t s);
hipError_t launch_gen_exact(const DevPlan &p, const GenPlan &g, bool mixed, bool all_lu, const uint64_t *keys,
                            const double2 *w, int64_t nkeys, const uint64_t *bits, int64_t B, uint32_t *flags,
                            void *setup, double *prob, double *amp, double *logp, unsigned long long *nterm,
                            hipEvent_t ev_mid, hipStream_t s, const DevTree *tree);
hipError_t prepare_gen();
// Device address of the no-allocation scratch on `device` (current), looked up
// once per device (k_noalloc.hip).
hipError_t noalloc_scratch(int device, void **ptr);
size_t raw_estimate_lds_bytes(const DevPlan &p, bool mixed);
size_t exact_lds_bytes(const DevPlan &p);
size_t raw_estimate_bwd_lds_bytes(const DevPlan &p, bool mixed);
size_t exact_bwd_lds_bytes(const DevPlan &p);

}  // namespace xf
