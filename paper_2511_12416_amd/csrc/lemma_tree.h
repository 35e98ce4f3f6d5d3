// Exact mode by a prefix tree over the term list.
//
// Under the determinant lemma with an unshifted base, a term with flip
// pattern N contributes w(N) det M_B det G[N, N] (Sec. IV-B Eq. 16-19 moved
// onto the base), where G is fixed per bitstring and block-diagonal over the
// spin blocks: G = I - 2H for one CPhase layer; G = I + 2T - 2H for two,
// with T = R'_1 from layer-0 to layer-1 positions (zero elsewhere: T^2 = 0,
// so det(I + 2T - 2H)[N, N] = det(I - 2(I - 2T)H)[N, N], the two-layer form
// that corrects the layer-1 rows by the pattern's layer-0 flips); G = I +
// 2TT - 2K for more than two (lemma_gen.h).  Every det G[N, N] is a
// principal minor of the same matrix, so the terms share work: ordering the flipped positions, a term's
// minor is the product of the pivots of Gaussian elimination in that order,
// and terms with a common prefix share its elimination (the recursion of
// Griffin and Tsatsomeros for all principal minors of a matrix, Linear
// Algebra Appl. 419 (2006), taken here four positions at a time).
//
// The tree (built once per plan on the host, shared by every bitstring): an
// anchor is a set of 4 l positions that is the prefix of some pattern; its
// matrix is the Schur complement G / G[anchor, anchor] on the positions its
// descendants still need, computed from its parent's by eliminating four
// positions (Gaussian elimination of a 4 x 4 block, then a rank-4 update); its
// prefix determinant is the parent's times det of that block.  A pattern
// hangs from its deepest anchor with at most four positions left, and costs a
// det of at most 4 x 4 of its anchor's matrix.
//
// Elimination in a fixed order can lose accuracy where a pivot is small; the
// kernel tracks the growth it allows (the largest |multiplier|^2 of the
// blocks' eliminations, and the largest |entry|^2 of any anchor matrix over
// the largest of G) and leaves every bitstring whose growth exceeds the
// plan's limit, or that meets a zero pivot, to the pattern pass (which
// factorises each pattern's r x r matrix on its own with partial pivoting).
// The patterns' own determinants (at most 4 x 4) use partial pivoting.
#pragma once
#include "lemma_gen.h"

namespace xf {
namespace {

// 1 / x for a normal, finite x > 0: the hardware reciprocal estimate
// refined by two Newton steps (each at least doubles the correct bits).
__device__ __forceinline__ double recip(double x) {
    double r = __builtin_amdgcn_rcp(x);
    double e = fma(-x, r, 1.0);
    r = fma(r, e, r);
    e = fma(-x, r, 1.0);
    return fma(r, e, r);
}

// Solves a x = b (b replaced by x) for a 4 x 4 complex a by Gaussian
// elimination in the given order (the tree's order: no row exchanges) and
// returns det a; 0 (and b unspecified) for a zero or non-finite pivot.  gl
// takes the largest |multiplier|^2, the growth the elimination allows.
__device__ __forceinline__ double2 solve4(double2 (&a)[4][4], double2 (&b)[4], double &gl) {
    double2 det = make_double2(1.0, 0.0);
    double2 inv[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        const double2 pv = a[c][c];
        const double n2 = cabs2(pv);
        if (!(n2 > 0.0 && n2 < 1e300)) return make_double2(0.0, 0.0);
        det = c_mul(det, pv);
        const double rb = recip(n2);
        inv[c] = make_double2(pv.x * rb, -pv.y * rb);
#pragma unroll
        for (int i = c + 1; i < 4; ++i) {
            const double2 l = c_mul(a[i][c], inv[c]);
            gl = fmax(gl, cabs2(l));
            const double2 nl = make_double2(-l.x, -l.y);
#pragma unroll
            for (int j = c + 1; j < 4; ++j) a[i][j] = c_fma(a[i][j], nl, a[c][j]);
            b[i] = c_fma(b[i], nl, b[c]);
        }
    }
#pragma unroll
    for (int c = 3; c >= 0; --c) {
        double2 v = b[c];
#pragma unroll
        for (int j = c + 1; j < 4; ++j) v = c_fma(v, make_double2(-a[c][j].x, -a[c][j].y), b[j]);
        b[c] = c_mul(v, inv[c]);
    }
    return det;
}

// A pattern in registers: its weight, then r and idx[0..2] in m0 and idx[3]
// in m1 (the byte layout of TreePat).
struct PatRegs {
    double2 w;
    uint32_t m0, m1;
};
__device__ __forceinline__ PatRegs load_pat(const DevTree &tr, uint32_t q) {
    const TreePat *t = tr.pat + q;
    PatRegs r;
    r.w = t->w;
    const uint2 m = *(const uint2 *)((const unsigned char *)t + 16);
    r.m0 = m.x;
    r.m1 = m.y;
    return r;
}

// One pattern: det of its r x r block of its anchor's matrix Q (row stride
// ld), times its anchor's prefix determinant, the base determinant and its
// weight, added exactly to acc.  Returns r.
__device__ __forceinline__ int tree_pattern(const PatRegs &tp, const double2 *Q, int ld, double2 dpre, double2 detB,
                                            FixAcc &acc) {
    const int r = (int)(tp.m0 & 0xFF);
    int idx[4];
#pragma unroll
    for (int u = 0; u < 3; ++u) idx[u] = (int)((tp.m0 >> (8 * (u + 1))) & 0xFF);
    idx[3] = (int)(tp.m1 & 0xFF);
    double2 a[4][4];
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int v = 0; v < 4; ++v)
            a[u][v] = (u < r && v < r) ? Q[idx[u] * ld + idx[v]] : make_double2(u == v ? 1.0 : 0.0, 0.0);
    const double2 d = small_det4(a, r);
    const double2 val = c_mul(tp.w, c_mul(detB, c_mul(dpre, d)));
    fix_add_double(acc.re, acc.bad, val.x);
    fix_add_double(acc.im, acc.bad, val.y);
    return r;
}

__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
    return v;
}

// LDS ordering between the phases of one wave (the workgroup is one wave,
// whose LDS accesses complete in issue order): a compiler fence, with no
// wait on the global loads prefetched for the next anchor.
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

// Evaluates the n staged patterns (a lane each): det of the 4 x 4 block
// (LU with partial pivoting) times the factor, added exactly to acc.
__device__ __forceinline__ void tree_flush(const double2 *St, const double2 *Fs, int n, FixAcc &acc) {
    const int lane = threadIdx.x;
    if (lane < n) {
        double2 a[4][4];
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
            for (int v = 0; v < 4; ++v) a[u][v] = St[lane * 16 + 4 * u + v];
        const double2 val = c_mul(Fs[lane], small_det4(a, 4));
        fix_add_double(acc.re, acc.bad, val.x);
        fix_add_double(acc.im, acc.bad, val.y);
    }
    wave_sync();
}

// 64 anchor records, one per lane (five words each), and the fields of one
// of them read back into every lane.
struct AncLanes {
    uint32_t w[5];
};
struct AncAt {
    uint32_t pat0, npat, roff;
    int level, nr, pnr;
    int j[4];
    int flags;   // kTreeLeaf, kTreePairFirst
};
// An anchor without children: its patterns are staged straight from its
// parent's matrix (no matrix of its own).  The first of two sibling leaves
// that one step takes together, a half-wave each (the next record is the
// other).
constexpr int kTreeLeaf = 1, kTreePairFirst = 2;
__device__ __forceinline__ void load_anchor_lanes(const DevTree &tr, int base, AncLanes &a) {
    // unconditional loads (clamped index), so that no branch holds back the
    // compiler's wait counts
    const int idx = base + (int)threadIdx.x;
    const uint32_t *q = (const uint32_t *)tr.anc + 5 * (size_t)(idx < tr.nanc ? idx : 0);
#pragma unroll
    for (int k = 0; k < 5; ++k) a.w[k] = q[k];
}
__device__ __forceinline__ AncAt anchor_at(const AncLanes &a, int lane) {
    uint32_t w[5];
#pragma unroll
    for (int k = 0; k < 5; ++k) w[k] = (uint32_t)__builtin_amdgcn_readlane((int)a.w[k], lane);
    AncAt r;
    r.pat0 = w[0];
    r.npat = w[1];
    r.roff = w[2];
    r.level = (int)(w[3] & 0xFF);
    r.nr = (int)((w[3] >> 8) & 0xFF);
    r.pnr = (int)((w[3] >> 16) & 0xFF);
    r.j[0] = (int)(w[3] >> 24);
    r.j[1] = (int)(w[4] & 0xFF);
    r.j[2] = (int)((w[4] >> 8) & 0xFF);
    r.j[3] = (int)((w[4] >> 16) & 0xFF);
    r.flags = (int)(w[4] >> 24);
    return r;
}

// Record idx of the two chunks held in the lanes (cur: base .. base + 63,
// nxt: the 64 after).
__device__ __forceinline__ AncAt anchor_of(const AncLanes &cur, const AncLanes &nxt, int base, int idx) {
    return idx < base + 64 ? anchor_at(cur, idx - base) : anchor_at(nxt, idx - base - 64);
}

// A step's global loads, issued one step ahead: the R index of this lane's
// column (lanes 0..63 of one anchor, or 0..31 and 32..63 of a pair) and the
// pattern of its staging slot (lane / 16 in the step's pattern list).
// Unconditional loads on clamped indices (each array has one element of
// padding).
struct StepLoads {
    int rr;
    PatRegs pp;
};
__device__ __forceinline__ StepLoads step_loads(const DevTree &tr, const AncAt &a, const AncAt &b, bool two,
                                                bool valid) {
    const int lane = threadIdx.x;
    const bool hb = two && lane >= 32;
    const int l = two ? (lane & 31) : lane;
    const uint32_t roff = hb ? b.roff : a.roff;
    const int nr = hb ? b.nr : a.nr;
    const uint32_t ri = valid ? roff + (uint32_t)min(l, max(nr - 1, 0)) : 0u;
    const int q = lane >> 4, na = (int)a.npat, nb = (int)b.npat;
    uint32_t pi = a.pat0 + (uint32_t)min(q, max(na - 1, 0));
    if (two && q >= na) pi = b.pat0 + (uint32_t)min(q - na, max(nb - 1, 0));
    StepLoads s;
    s.rr = tr.ridx[ri];
    s.pp = load_pat(tr, valid ? pi : 0u);
    return s;
}

// The matrix of an anchor A with children, from its parent's (level
// A.level - 1): T = P[J, J]^-1 P[J, R] (a column per lane; every lane
// factorises the same block) into Tb, its R indices into sR[0], the prefix
// determinant into Dl[A.level], then Q = P[R, R] - P[R, J] T (an entry per
// lane; e / nr by a multiply, exact for e < nr^2 <= 1024, nr <= 32) into the
// level's slot.  rr: this lane's R index (lanes < A.nr).
__device__ __forceinline__ void tree_anchor_matrix(const DevTree &tr, double2 *S, double2 *Tb, double2 *Dl,
                                                   int (*sR)[kTreeMaxM], const AncAt &A, int rr, double &gl,
                                                   double &grow, bool &bad) {
    const int lane = threadIdx.x;
    const int lv = A.level, nr = A.nr, pnr = A.pnr;
    const double2 *P = S + tr.slot[lv - 1];
    double2 *Q = S + tr.slot[lv];
    if (lane < max(nr, 1)) {
        double2 m4[4][4], x[4];
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
            for (int v = 0; v < 4; ++v) m4[u][v] = P[A.j[u] * pnr + A.j[v]];
#pragma unroll
        for (int u = 0; u < 4; ++u) x[u] = lane < nr ? P[A.j[u] * pnr + rr] : make_double2(0.0, 0.0);
        const double2 dJ = solve4(m4, x, gl);
        bad |= dJ.x == 0.0 && dJ.y == 0.0;
        if (lane < nr) {
            sR[0][lane] = rr;
#pragma unroll
            for (int u = 0; u < 4; ++u) Tb[u * tr.maxr + lane] = x[u];
        }
        if (lane == 0) Dl[lv] = c_mul(Dl[lv - 1], dJ);
    }
    wave_sync();
    const uint32_t mg = ((1u << 20) + (uint32_t)nr - 1) / (uint32_t)max(nr, 1);
    for (int e = lane; e < nr * nr; e += 64) {
        const int ii = (int)(((uint32_t)e * mg) >> 20), jj = e - ii * nr;
        const int ri = sR[0][ii], rj = sR[0][jj];
        double2 sv = P[ri * pnr + rj];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const double2 c = P[ri * pnr + A.j[u]];
            sv = c_fma(sv, make_double2(-c.x, -c.y), Tb[u * tr.maxr + jj]);
        }
        Q[e] = sv;
        grow = fmax(grow, cabs2(sv));
    }
    wave_sync();
}

// One anchor record read directly (uniform index).
__device__ __forceinline__ AncAt anchor_direct(const DevTree &tr, uint32_t x) {
    const uint32_t *q = (const uint32_t *)tr.anc + 5 * (size_t)x;
    uint32_t w[5];
#pragma unroll
    for (int k = 0; k < 5; ++k) w[k] = q[k];
    AncAt r;
    r.pat0 = w[0];
    r.npat = w[1];
    r.roff = w[2];
    r.level = (int)(w[3] & 0xFF);
    r.nr = (int)((w[3] >> 8) & 0xFF);
    r.pnr = (int)((w[3] >> 16) & 0xFF);
    r.j[0] = (int)(w[3] >> 24);
    r.j[1] = (int)(w[4] & 0xFF);
    r.j[2] = (int)((w[4] >> 8) & 0xFF);
    r.j[3] = (int)((w[4] >> 16) & 0xFF);
    r.flags = (int)(w[4] >> 24);
    return r;
}

// One wave per (bitstring, part) item (grid-stride): part pi of `parts`
// covers the plan's parts pa .. pb - 1, a run of the depth-first anchor
// order, which it walks after recomputing its first anchor's ancestors (the
// root's patterns go with the first part).  Takes the bitstrings whose setup
// succeeded with unshifted bases (flag 0, shift 0).  With one part: on
// success writes p, A and log p and sets the flag to kEntryTree, so that the
// pattern pass skips them; otherwise leaves the flag for the pattern pass.
// With several: writes each part's exact partial sum and its failure bit to
// part[item], for k_gen_tree_reduce.  LDS: tr.lds bytes (the levels'
// matrices, two T buffers, the prefix determinants and the staged patterns).
// The anchor records come 64 at a time into the lanes' registers (the next
// 64 loaded while these are used); each step's R indices and first four
// patterns are loaded one step ahead.  A step is one anchor, or two sibling
// leaves (a half-wave each), whose patterns' blocks are formed from the
// parent's matrix without a matrix of their own.  An anchor's patterns are
// copied, as identity-padded 4 x 4 blocks with their factors, into a stage
// that is evaluated kTreeStage at a time (a lane each), so that the
// determinants run on full waves although an anchor has few patterns.
template <bool MULTI>
__global__ void __launch_bounds__(64)
k_gen_tree(DevPlan p, GenPlan g, DevTree tr, int64_t nb, int parts, uint32_t *__restrict__ flags,
           const double2 *__restrict__ hbuf, const GenRec *__restrict__ rec, double *__restrict__ prob,
           double *__restrict__ amp, double *__restrict__ logp, unsigned long long *nterm,
           uint64_t *__restrict__ part) {
    static_assert(sizeof(TreeAnchor) == 20, "anchor records are five words");
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ int sR[2][kTreeMaxM];
    double2 *S = (double2 *)smem;
    double2 *Tb = S + tr.toff;
    double2 *Dl = S + tr.doff;
    double2 *St = S + tr.soff;                      // staged blocks, 16 entries each
    double2 *Fs = St + 16 * kTreeStage;             // their factors
    const int lane = threadIdx.x;
    const int M = tr.M;
    Work wk;
    unsigned long long done = 0;
    for (int64_t item = blockIdx.x; item < nb * (int64_t)parts; item += gridDim.x) {
        const int64_t i = item / parts;
        const int pi = (int)(item - i * parts);
        if (flags[i] != 0) continue;
        const uint64_t sh0 = rec[i].shift[0], sh1 = rec[i].shift[1];
        if (sh0 | sh1) continue;
        const double2 detB = rec[i].det;
        const double2 *Hg = hbuf + (size_t)i * g.hsize;
        // this item's anchors: a run of the depth-first order (the plan's
        // parts pa .. pb - 1), after its first anchor's ancestors
        const int pa = (pi * tr.nparts) / parts, pb = ((pi + 1) * tr.nparts) / parts;
        const int lo = (int)tr.pstart[pa], hi = (int)tr.pstart[pb];
        AncLanes cur, nxt;
        load_anchor_lanes(tr, lo, cur);
        load_anchor_lanes(tr, lo + 64, nxt);
        // G on the tree's positions (zero across blocks)
        double gmax = 0.0;
        for (int e = lane; e < M * M; e += 64) {
            const int a = e / M, b = e - a * M;
            const int ca = tr.rpos[a], cb = tr.rpos[b];
            const int blk = ca >> 8;
            double2 v = make_double2(0.0, 0.0);
            if (blk == (cb >> 8)) {
                const int pa = ca & 0xFF, pb = cb & 0xFF;
                const double2 h = Hg[g.hoff[blk] + pa * g.hld[blk] + pb];
                v = make_double2((a == b ? 1.0 : 0.0) - 2.0 * h.x, -2.0 * h.y);
                if constexpr (MULTI) {
                    const double2 t = g.TT[((size_t)blk * 64 + pa) * 64 + pb];
                    v.x += 2.0 * t.x;
                    v.y += 2.0 * t.y;
                } else if (p.L == 2 && pa >= g.kb0[blk] && pb < g.kb0[blk]) {
                    // two layers: T = R'_1 from layer-0 to layer-1 positions
                    const uint8_t *act = g.act + blk * kGenMaxKb;
                    const double2 t = p.R1[(size_t)act[pa] * p.n + act[pb]];
                    v.x += 2.0 * t.x;
                    v.y += 2.0 * t.y;
                }
            }
            S[e] = v;
            gmax = fmax(gmax, cabs2(v));
        }
        if (lane == 0) Dl[0] = make_double2(1.0, 0.0);
        wave_sync();
        FixAcc acc;
        double grow = 0.0, gl = 0.0;
        bool bad = false;
        unsigned long long rank = 0, flops = 0;
        int nst = 0;   // patterns staged
        for (int q = lane; q < (pa == 0 ? tr.nroot : 0); q += 64) {
            const int r = tree_pattern(load_pat(tr, q), S, M, Dl[0], detB, acc);
            rank += r;
            flops += lu_flops(r) + 18;
        }
        // (the R index and pattern loads are unconditional, on clamped
        // indices: both arrays hold at least one element)
        int base = lo;
        AncAt A0 = anchor_of(cur, nxt, base, lo);
        AncAt A1 = anchor_of(cur, nxt, base, hi - lo > 1 ? lo + 1 : lo);
        bool two = hi - lo > 1 && (A0.flags & kTreePairFirst);
        StepLoads ld = step_loads(tr, A0, A1, two, hi > lo);
        // the ancestors' matrices (their patterns belong to earlier parts)
        for (int l = 1; l < (hi > lo ? A0.level : 0); ++l) {
            const AncAt C = anchor_direct(tr, tr.pchain[(size_t)pa * 8 + l]);
            const int rc = tr.ridx[C.roff + min(lane, max(C.nr - 1, 0))];
            tree_anchor_matrix(tr, S, Tb, Dl, sR, C, rc, gl, grow, bad);
        }
        for (int st = lo; st < hi;) {
            // the next step's records (the chunks move on when it starts past
            // the first; st < base + 64 holds at every step) and loads
            const int ns = st + (two ? 2 : 1);
            if (ns >= base + 64) {
                cur = nxt;
                base += 64;
                load_anchor_lanes(tr, base + 64, nxt);
            }
            const bool more = ns < hi;
            const AncAt B0 = anchor_of(cur, nxt, base, more ? ns : base);
            const AncAt B1 = anchor_of(cur, nxt, base, ns + 1 < hi ? ns + 1 : (more ? ns : base));
            const bool twoB = ns + 1 < hi && (B0.flags & kTreePairFirst);
            const StepLoads ldB = step_loads(tr, B0, B1, twoB, more);

            const int lv = A0.level, pnr = A0.pnr;
            const double2 *P = S + tr.slot[lv - 1];
            if (A0.flags & kTreeLeaf) {
                // one leaf, or two sibling leaves (a half-wave each): T for
                // each, then its patterns' blocks of P[R, R] - P[R, J] T
                // staged directly
                const int hb = (two && lane >= 32) ? 1 : 0;
                const int l = two ? (lane & 31) : lane;
                const int nr = hb ? A1.nr : A0.nr;
                int J[4];
#pragma unroll
                for (int u = 0; u < 4; ++u) J[u] = hb ? A1.j[u] : A0.j[u];
                if ((hb == 0 || two) && l < max(nr, 1)) {
                    double2 m4[4][4], x[4];
#pragma unroll
                    for (int u = 0; u < 4; ++u)
#pragma unroll
                        for (int v = 0; v < 4; ++v) m4[u][v] = P[J[u] * pnr + J[v]];
#pragma unroll
                    for (int u = 0; u < 4; ++u) x[u] = l < nr ? P[J[u] * pnr + ld.rr] : make_double2(0.0, 0.0);
                    const double2 dJ = solve4(m4, x, gl);
                    bad |= dJ.x == 0.0 && dJ.y == 0.0;
                    if (l < nr) {
                        sR[hb][l] = ld.rr;
#pragma unroll
                        for (int u = 0; u < 4; ++u) Tb[(hb * 4 + u) * tr.maxr + l] = x[u];
                    }
                    if (l == 0) Dl[kTreeLevels + hb] = c_mul(Dl[lv - 1], dJ);
                }
                wave_sync();
                const int na = (int)A0.npat, total = na + (two ? (int)A1.npat : 0);
                for (int q0 = 0; q0 < total; q0 += 4) {
                    const int cnt = min(4, total - q0);
                    if (nst + cnt > kTreeStage) {
                        wave_sync();
                        tree_flush(St, Fs, nst, acc);
                        nst = 0;
                    }
                    const int ql = lane >> 4, e = lane & 15, u = e >> 2, v = e & 3;
                    if (ql < cnt) {
                        const int q = q0 + ql;
                        const int qb = q >= na ? 1 : 0;
                        const PatRegs t =
                            q0 == 0 ? ld.pp : load_pat(tr, qb ? A1.pat0 + (uint32_t)(q - na) : A0.pat0 + (uint32_t)q);
                        const int r = (int)(t.m0 & 0xFF);
                        const uint64_t mm = (uint64_t)t.m0 | ((uint64_t)t.m1 << 32);
                        const int iu = (int)((mm >> (8 * (u + 1))) & 0xFF), iv = (int)((mm >> (8 * (v + 1))) & 0xFF);
                        double2 val = make_double2(u == v ? 1.0 : 0.0, 0.0);
                        if (u < r && v < r) {
                            const int ri = sR[qb][iu], rj = sR[qb][iv];
                            val = P[ri * pnr + rj];
#pragma unroll
                            for (int w = 0; w < 4; ++w) {
                                const double2 c = P[ri * pnr + (qb ? A1.j[w] : A0.j[w])];
                                val = c_fma(val, make_double2(-c.x, -c.y), Tb[(qb * 4 + w) * tr.maxr + iv]);
                            }
                            grow = fmax(grow, cabs2(val));
                        }
                        St[(nst + ql) * 16 + e] = val;
                        if (e == 0) {
                            Fs[nst + ql] = c_mul(t.w, c_mul(detB, Dl[kTreeLevels + qb]));
                            rank += 4 * lv + r;
                            flops += lu_flops(r) + 18 + 32ull * r * r;
                        }
                    }
                    nst += cnt;
                }
                if (lane == 0)
                    flops += lu_flops(4) + 128ull * A0.nr + 6 + (two ? lu_flops(4) + 128ull * A1.nr + 6 : 0ull);
            } else {
                const int nr = A0.nr;
                double2 *Q = S + tr.slot[lv];
                tree_anchor_matrix(tr, S, Tb, Dl, sR, A0, ld.rr, gl, grow, bad);
                // stage the anchor's patterns, four per pass (16 lanes each:
                // one entry of the 4 x 4 block, identity past r) with their
                // factors w det M_B dpre; evaluate the stage when it is full
                const double2 dpre = Dl[lv];
                for (int q0 = 0; q0 < (int)A0.npat; q0 += 4) {
                    const int cnt = min(4, (int)A0.npat - q0);
                    if (nst + cnt > kTreeStage) {
                        wave_sync();
                        tree_flush(St, Fs, nst, acc);
                        nst = 0;
                    }
                    const int ql = lane >> 4, e = lane & 15, u = e >> 2, v = e & 3;
                    if (ql < cnt) {
                        const PatRegs t = q0 == 0 ? ld.pp : load_pat(tr, A0.pat0 + q0 + ql);
                        const int r = (int)(t.m0 & 0xFF);
                        const uint64_t mm = (uint64_t)t.m0 | ((uint64_t)t.m1 << 32);
                        const int iu = (int)((mm >> (8 * (u + 1))) & 0xFF), iv = (int)((mm >> (8 * (v + 1))) & 0xFF);
                        St[(nst + ql) * 16 + e] =
                            (u < r && v < r) ? Q[iu * nr + iv] : make_double2(u == v ? 1.0 : 0.0, 0.0);
                        if (e == 0) {
                            Fs[nst + ql] = c_mul(t.w, c_mul(detB, dpre));
                            rank += 4 * lv + r;
                            flops += lu_flops(r) + 18;
                        }
                    }
                    nst += cnt;
                }
                if (lane == 0) flops += lu_flops(4) + 128ull * nr + 32ull * nr * nr + 6;
            }
            wave_sync();
            A0 = B0;
            A1 = B1;
            two = twoB;
            ld = ldB;
            st = ns;
        }
        wave_sync();
        tree_flush(St, Fs, nst, acc);
        const double gm = wave_max(gmax), gr = wave_max(grow), ml = wave_max(gl);
        const bool fail = __ballot(bad) != 0 || !(gr <= tr.growth2 * gm) || !(ml <= tr.growth2);
        if (fail && parts == 1) continue;   // the pattern pass takes it
        fix_wave_sum(acc.re);
        fix_wave_sum(acc.im);
        const bool accbad = __ballot(acc.bad) != 0;
        if (!fail) {
            wk.rank += rank;
            wk.flops += flops;
        }
        if (lane == 0) {
            const uint64_t words[kAccWords] = {acc.re.w0, acc.re.w1, (uint64_t)acc.re.w2, acc.im.w0,
                                               acc.im.w1, (uint64_t)acc.im.w2,
                                               (accbad ? 1ull : 0ull) | (fail ? 2ull : 0ull)};
            if (parts == 1) {
                write_result(i, acc_value(words), 1.0, prob, amp, logp);
                flags[i] = kEntryTree;
                wk.terms += (unsigned)tr.npat;
                ++done;
            } else {
                // a part's exact partial sum; bit 1 of the last word: this
                // part's growth or pivots fail (k_gen_tree_reduce)
#pragma unroll
                for (int w = 0; w < kAccWords; ++w) part[(size_t)item * 8 + w] = words[w];
            }
        }
    }
    flush_work(wk, nterm);
    if (nterm && lane == 0 && done) atomicAdd(nterm + 7, done);
}

// The sum of the parts of each bitstring the tree kernel took in `parts`
// parts (in part order; the words are exact integers), one thread per
// bitstring: p, A and log p written and the flag set to kEntryTree, unless
// a part failed (then the pattern pass takes the bitstring).
__global__ void k_gen_tree_reduce(int64_t nb, int parts, int npat, uint32_t *__restrict__ flags,
                                  const GenRec *__restrict__ rec, const uint64_t *__restrict__ part,
                                  double *__restrict__ prob, double *__restrict__ amp, double *__restrict__ logp,
                                  unsigned long long *nterm) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nb || flags[i] != 0 || (rec[i].shift[0] | rec[i].shift[1])) return;
    Fix192 R, I;
    uint64_t bad = 0;
    for (int j = 0; j < parts; ++j) {
        const uint64_t *q = part + ((size_t)i * parts + j) * 8;
        fix_add(R, q[0], q[1], (int64_t)q[2]);
        fix_add(I, q[3], q[4], (int64_t)q[5]);
        bad |= q[6];
    }
    if (bad & 2) return;
    const uint64_t acc[kAccWords] = {R.w0, R.w1, (uint64_t)R.w2, I.w0, I.w1, (uint64_t)I.w2, bad & 1};
    write_result(i, acc_value(acc), 1.0, prob, amp, logp);
    flags[i] = kEntryTree;
    if (nterm) {
        atomicAdd(nterm, (unsigned long long)npat);
        atomicAdd(nterm + 7, 1ull);
    }
}

}  // namespace
}  // namespace xf
