// Host side of the C ABI declared in include/xf.h: argument validation, the
// FP64 plan precompute (absorbed d_0 phases, low-rank factors, sampling
// table, bit-compressed flip keys, exact-mode term list), the matrix
// exponential helpers, and the kernel launches.
//
// Built with -ffp-contract=off on the baseline x86-64 ISA so that the sampling
// table is computed operation by operation as its definition states.
#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <cmath>
#include <complex>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "../../include/xf.h"
#include "xf_internal.h"

using cd = std::complex<double>;

namespace {

thread_local std::string g_err;

xf_status fail(xf_status s, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return s;
}

xf_status ok() {
    g_err.clear();
    return XF_OK;
}

// ---------------------------------------------------------------------------
// small dense complex helpers (row-major)
// ---------------------------------------------------------------------------

void matmul(const cd *A, const cd *B, cd *C, int p, int q, int r) {
    for (int i = 0; i < p; ++i)
        for (int j = 0; j < r; ++j) {
            cd acc = 0.0;
            for (int l = 0; l < q; ++l) acc += A[(size_t)i * q + l] * B[(size_t)l * r + j];
            C[(size_t)i * r + j] = acc;
        }
}

double norm1(const std::vector<cd> &A, int n) {
    double best = 0.0;
    for (int j = 0; j < n; ++j) {
        double s = 0.0;
        for (int i = 0; i < n; ++i) s += std::abs(A[(size_t)i * n + j]);
        best = std::max(best, s);
    }
    return best;
}

// exp(A) by scaling and squaring with a degree-24 Taylor polynomial on
// A / 2^s, ||A / 2^s||_1 <= 1/2 (truncation below 1e-30 relative).
std::vector<cd> expm(const std::vector<cd> &A, int n) {
    const double nrm = norm1(A, n);
    int s = 0;
    if (nrm > 0.5) s = (int)std::ceil(std::log2(nrm / 0.5));
    const double sc = std::ldexp(1.0, -s);
    std::vector<cd> X(A.size()), E((size_t)n * n, 0.0), term((size_t)n * n, 0.0), tmp((size_t)n * n);
    for (size_t i = 0; i < A.size(); ++i) X[i] = A[i] * sc;
    for (int i = 0; i < n; ++i) E[(size_t)i * n + i] = 1.0, term[(size_t)i * n + i] = 1.0;
    for (int d = 1; d <= 24; ++d) {
        matmul(term.data(), X.data(), tmp.data(), n, n, n);
        for (size_t i = 0; i < tmp.size(); ++i) term[i] = tmp[i] / (double)d;
        for (size_t i = 0; i < E.size(); ++i) E[i] += term[i];
    }
    for (int i = 0; i < s; ++i) {
        matmul(E.data(), E.data(), tmp.data(), n, n, n);
        E.swap(tmp);
    }
    return E;
}

bool finite_all(const double *p, size_t cnt) {
    for (size_t i = 0; i < cnt; ++i)
        if (!std::isfinite(p[i])) return false;
    return true;
}

// ---------------------------------------------------------------------------
// device buffers
// ---------------------------------------------------------------------------

struct DevBuf {
    void *p = nullptr;
    size_t bytes = 0;
};

xf_status dev_upload(DevBuf &b, const void *src, size_t bytes) {
    if (bytes == 0) bytes = 16;
    if (b.bytes < bytes) {
        if (b.p) hipFree(b.p);
        b.p = nullptr;
        b.bytes = 0;
        if (hipMalloc(&b.p, bytes) != hipSuccess) return fail(XF_ENOMEM, "hipMalloc(%zu) failed", bytes);
        b.bytes = bytes;
    }
    if (src && hipMemcpy(b.p, src, bytes, hipMemcpyHostToDevice) != hipSuccess)
        return fail(XF_EDEVICE, "hipMemcpy to device failed");
    return XF_OK;
}

void dev_free(DevBuf &b) {
    if (b.p) hipFree(b.p);
    b.p = nullptr;
    b.bytes = 0;
}

struct DeviceGuard {
    int prev = -1;
    bool okay = false;
    explicit DeviceGuard(int dev) {
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        okay = hipSetDevice(dev) == hipSuccess;
    }
    ~DeviceGuard() {
        if (prev >= 0) hipSetDevice(prev);
    }
};

}  // namespace

// Rotation layers of a plan (CPhase layers + 1).
constexpr int kMaxRot = 65;

struct xf_plan {
    int device = 0;
    int n = 0, n_rot = 0, k = 0, m = 0, L = 0, G = 4;
    xf_precision precision = XF_FP64;
    std::vector<double> rot;      // [n_rot][n][n][2]
    std::vector<int32_t> pairs;   // [k][2]
    std::vector<int32_t> layer;   // [k]
    std::vector<double> theta;    // [k]
    std::vector<int> C;           // occupied input modes
    // flip-pattern keys
    int keykind = 0, keybits = 0, off1 = 0;
    std::vector<uint8_t> keymode;     // [64]
    std::vector<uint64_t> gkey;       // [k]
    std::vector<uint64_t> gmode;      // [k][2]
    std::vector<uint8_t> gneg;        // [k]
    // device state
    DevBuf dP, dPhi0, dA1, dA2, dQ, dR1, fPhi0, fA1, fA2, fQ, fR1;
    DevBuf dkeymode, dT, dgkey, dgmode, dglayer, dgneg, dnterm;
    DevBuf dxkeys, dxw, dxdw;         // exact-mode term list (+ angle derivatives of the weights)
    // general determinant-lemma evaluation: blocks of modes and their active lists
    xf::GenPlan gen{};
    DevBuf dgcol, dgact, dgpos0, dgpos1, dgblk, dgkbt, dggpos, dflags;
    DevBuf dgGA, dgHC, dgTT;          // more than two CPhase layers: the factors of each block's positions
    DevBuf dgsetup;                   // general lemma: per-bitstring H and base records
    std::vector<uint16_t> hkbt;       // host copy of the key-bit table of the general lemma
    // exact mode: the term list's prefix tree (lemma_tree.h), built with it
    DevBuf dtanc, dtridx, dtpat, dtrpos, dtpart, dtchain;
    xf::DevTree tree{};
    bool has_tree = false;
    // the tree's position order, kept while the set of flip patterns (not
    // their weights) stays the same
    std::vector<uint16_t> tree_codes;
    uint64_t tree_key = 0;
    double tree_growth = 1e4;         // growth accepted along the tree
    int last_gen = 0;                 // the last xf_probabilities call used the general lemma kernel
    int64_t nxterms = -1;             // -1: not built for the current parameters
    xf_evaluation evaluation = XF_EVAL_AUTO;
    double mixed_cond = 100.0;        // XF_MIXED: kappa_1 bound of bases formed in FP32
    int last_lemma = 0;               // the last xf_probabilities call used the determinant lemma
    int last_bwd_lemma = 0;           // the last xf_log_prob_backward call used the determinant lemma
    int last_bwd_reused = 0;          // ... and took the forward call's patterns from the workspace
    // determinant-lemma workspace: per-bitstring regions of (pattern, count) entries
    DevBuf dekey, decnt, decount;
    uint64_t entry_budget = 16ull << 30;  // bytes of workspace the chunking aims at
    // the last Raw Estimate forward call whose patterns the workspace still
    // holds (one-layer lemma kernels, one chunk), for xf_plan_set_reuse_samples
    bool reuse_samples = false;
    bool fwd_valid = false;
    const void *fwd_bits = nullptr;
    int64_t fwd_B = 0, fwd_t = 0;
    uint64_t fwd_seed = 0;
    // timing of the last call: ev[0] start, then per chunk (mid, end) of the
    // two lemma kernels, or one end event for a fused kernel
    std::vector<hipEvent_t> ev;
    int nev = 0;
    bool xterms_have_dw = false;
    // host copies of the factors, for the backward chain rule
    std::vector<std::vector<cd>> Rp;  // R'_l = R_l D0_{l-1} (R'_0 = R_0), n x n each
    std::vector<std::vector<cd>> d0;  // diagonal of D0_{l-1} for l >= 1 (index l)
    std::vector<cd> hPhi0;            // n x m
    DevBuf dpart, dgsum;              // backward scratch: per-workgroup partials, reduced sums
};

namespace {

bool plan_valid(const xf_plan *p) { return p != nullptr && p->n > 0; }

// Validates a circuit description (shared by create / set_params).
xf_status check_params(int n, int n_rot, const double *rot, int k, const double *theta) {
    if (!finite_all(rot, (size_t)n_rot * n * n * 2)) return fail(XF_EINVAL, "rotation contains NaN/Inf");
    for (int l = 0; l < n_rot; ++l) {
        const double *U = rot + (size_t)l * n * n * 2;
        double worst = 0.0;
        for (int i = 0; i < n; ++i)
            for (int j = 0; j < n; ++j) {
                cd acc = 0.0;
                for (int r = 0; r < n; ++r) {
                    const cd a(U[2 * ((size_t)r * n + i)], U[2 * ((size_t)r * n + i) + 1]);
                    const cd b(U[2 * ((size_t)r * n + j)], U[2 * ((size_t)r * n + j) + 1]);
                    acc += std::conj(a) * b;
                }
                worst = std::max(worst, std::abs(acc - (i == j ? 1.0 : 0.0)));
            }
        if (worst > 1e-10) return fail(XF_EINVAL, "rotation layer %d is not unitary (max |U^H U - I| = %.3g)", l, worst);
    }
    if (k > 0 && !finite_all(theta, (size_t)k)) return fail(XF_EINVAL, "theta contains NaN/Inf");
    for (int j = 0; j < k; ++j)
        if (!(std::fabs(theta[j]) < 2.0 * M_PI)) return fail(XF_EINVAL, "|theta[%d]| must be < 2 pi", j);
    return XF_OK;
}

// Sampling table (definition in xf.h): T[a][j] = min(floor(2^32 (1 - S)), 2^32 - 1),
// S = prod_{i=a..j} (1 - p_i), p_i = sin(|theta_i|/4) / (sin(|theta_i|/4) + cos(|theta_i|/4)).
std::vector<uint32_t> sampling_table(const std::vector<double> &theta) {
    const int k = (int)theta.size();
    std::vector<double> p(k);
    for (int j = 0; j < k; ++j) {
        const double s = std::sin(std::fabs(theta[j]) / 4.0);
        const double c = std::cos(std::fabs(theta[j]) / 4.0);
        p[j] = s / (s + c);
    }
    std::vector<uint32_t> T((size_t)k * k, 0u);
    for (int a = 0; a < k; ++a) {
        double S = 1.0;
        for (int j = a; j < k; ++j) {
            S = S * (1.0 - p[j]);
            const double f = 1.0 - S;
            const double v = std::floor(f * 4294967296.0);
            T[(size_t)a * k + j] = v >= 4294967295.0 ? 0xFFFFFFFFu : (uint32_t)v;
        }
    }
    return T;
}

double extent_of(const std::vector<double> &theta) {
    double xi = 1.0;
    for (double th : theta) {
        const double f = std::cos(std::fabs(th) / 4.0) + std::sin(std::fabs(th) / 4.0);
        xi *= f * f;
    }
    return xi;
}

// Blocks of modes for the general lemma evaluation: the connected components
// of the union of the rotation layers' nonzero patterns (every layer is then
// block-diagonal over them); two components give two blocks, any other count
// one block of all modes.  Per block: its input columns, the modes each CPhase
// layer touches in it, and their positions.
xf_status refresh_gen(xf_plan *P) {
    const int n = P->n, m = P->m;
    std::vector<int> parent(n);
    for (int i = 0; i < n; ++i) parent[i] = i;
    auto find = [&](int x) {
        while (parent[x] != x) x = parent[x] = parent[parent[x]];
        return x;
    };
    for (int l = 0; l < P->n_rot; ++l)
        for (int r = 0; r < n; ++r)
            for (int c = 0; c < n; ++c) {
                const double *z = &P->rot[2 * ((size_t)l * n * n + (size_t)r * n + c)];
                if (z[0] != 0.0 || z[1] != 0.0) parent[find(r)] = find(c);
            }
    std::vector<int> roots;
    for (int i = 0; i < n; ++i)
        if (find(i) == i) roots.push_back(i);
    xf::GenPlan &g = P->gen;
    g = xf::GenPlan{};
    g.nblk = roots.size() == 2 ? 2 : 1;
    const int L = P->L;
    const bool multi = L >= 3;
    g.multi = multi ? 1 : 0;
    std::vector<std::pair<int, int>> apos[2];   // (layer, mode) of each block's positions
    std::vector<int8_t> blk(128, 0), pos0(128, -1), pos1(128, -1);
    for (int q = 0; q < n; ++q) blk[q] = (int8_t)(g.nblk == 2 && find(q) == roots[1] ? 1 : 0);
    std::vector<uint8_t> col(2 * 32, 0), act(2 * 64, 0);
    bool fits = true;
    int hoff = 0, r1 = 0;
    for (int b = 0; b < g.nblk; ++b) {
        g.bmask[b][0] = g.bmask[b][1] = 0;
        for (int q = 0; q < n; ++q)
            if (blk[q] == b) g.bmask[b][q >> 6] |= 1ull << (q & 63);
        int mb = 0;
        for (int a = 0; a < m; ++a)
            if (blk[P->C[a]] == b) {
                if (mb < 32) col[b * 32 + mb] = (uint8_t)a;
                ++mb;
            }
        g.mb[b] = mb;
        // active positions: (CPhase layer, mode) pairs of the block, by layer then mode
        std::vector<std::vector<int>> al(std::max(L, 1));
        for (int j = 0; j < P->k; ++j)
            for (int side = 0; side < 2; ++side) {
                const int q = P->pairs[2 * j + side];
                if (blk[q] == b) al[P->layer[j]].push_back(q);
            }
        int kb = 0;
        for (auto &v : al) {
            std::sort(v.begin(), v.end());
            v.erase(std::unique(v.begin(), v.end()), v.end());
            kb += (int)v.size();
        }
        g.kb0[b] = multi ? kb : (int)al[0].size();
        g.kb[b] = kb;
        if (mb > 32 || kb > 64) fits = false;
        int at = 0;
        for (int l = 0; l < (int)al.size(); ++l)
            for (int q : al[l]) {
                if (at < 64) {
                    act[b * 64 + at] = (uint8_t)q;
                    if (l == 0) pos0[q] = (int8_t)at;
                    if (l == 1) pos1[q] = (int8_t)at;
                    apos[b].push_back({l, q});
                }
                ++at;
            }
        g.hoff[b] = hoff;
        g.hld[b] = g.kb[b] | 1;
        hoff += g.kb[b] * g.hld[b];
        g.r1off[b] = r1;
        r1 += multi ? kb * kb : g.kb0[b] * (g.kb[b] - g.kb0[b]);
    }
    g.hsize = hoff;
    g.r1size = r1;
    // key-bit table: a compressed key bit flips one (layer, mode); a
    // trajectory bit flips the two modes of gate j in its layer
    std::vector<uint16_t> kbt(128, 0xFFFF);
    auto code = [&](int layer, int q) -> uint16_t {
        if (multi) {
            const auto &v = apos[blk[q]];
            for (size_t i = 0; i < v.size(); ++i)
                if (v[i].first == layer && v[i].second == q) return (uint16_t)((blk[q] << 8) | i);
            return 0xFFFF;
        }
        const int ps = layer == 0 ? pos0[q] : pos1[q];
        return ps < 0 ? 0xFFFF : (uint16_t)((blk[q] << 8) | ps);
    };
    std::vector<uint16_t> gpos(128, 0xFFFF);
    for (int j = 0; j < P->k && j < 64; ++j)
        for (int side = 0; side < 2; ++side) gpos[2 * j + side] = code(P->layer[j], P->pairs[2 * j + side]);
    if (P->keykind == 0) {
        for (int i = 0; i < P->keybits && i < 64; ++i) kbt[2 * i] = code(i < P->off1 ? 0 : 1, P->keymode[i]);
    } else if (P->keykind == 1) {
        kbt = gpos;
    }
    if (!fits) g.nblk = 0;   // the general evaluation does not apply
    xf_status st;
    if (multi && fits) {
        // V(x) = R'_L W_{L-1} R'_{L-1} ... W_0 R'_0 with W_l = I - 2 E_l: for the
        // position q = (l, a) of a block, GA[:, q] = (R'_L ... R'_{l+1})[:, a],
        // HC[q, :] = (R'_l ... R'_0)[a, C], and for positions q = (l, a),
        // q' = (l', a') with l > l', TT[q, q'] = (R'_l ... R'_{l'+1})[a, a'].
        const auto &R = P->Rp;
        const int G = P->G;
        auto mv = [&](const std::vector<cd> &A, const std::vector<cd> &v) {
            std::vector<cd> o(n, 0.0);
            for (int r = 0; r < n; ++r)
                for (int c = 0; c < n; ++c) o[r] += A[(size_t)r * n + c] * v[c];
            return o;
        };
        auto vm = [&](const std::vector<cd> &v, const std::vector<cd> &A) {
            std::vector<cd> o(n, 0.0);
            for (int r = 0; r < n; ++r)
                for (int c = 0; c < n; ++c) o[c] += v[r] * A[(size_t)r * n + c];
            return o;
        };
        std::vector<double> GA((size_t)2 * n * 64 * 2, 0.0), HC((size_t)2 * 64 * G * 2, 0.0),
            TT((size_t)2 * 64 * 64 * 2, 0.0);
        for (int b = 0; b < g.nblk; ++b)
            for (size_t q = 0; q < apos[b].size(); ++q) {
                const int l = apos[b][q].first, a = apos[b][q].second;
                std::vector<cd> v(n, 0.0);
                v[a] = 1.0;
                for (int j = l + 1; j <= L; ++j) {
                    v = mv(R[j], v);
                    if (j < L)
                        for (size_t q2 = 0; q2 < apos[b].size(); ++q2)
                            if (apos[b][q2].first == j) {
                                const cd z = v[apos[b][q2].second];
                                TT[2 * (((size_t)b * 64 + q2) * 64 + q)] = z.real();
                                TT[2 * (((size_t)b * 64 + q2) * 64 + q) + 1] = z.imag();
                            }
                }
                for (int r = 0; r < n; ++r) {
                    GA[2 * (((size_t)b * n + r) * 64 + q)] = v[r].real();
                    GA[2 * (((size_t)b * n + r) * 64 + q) + 1] = v[r].imag();
                }
                std::vector<cd> u(n, 0.0);
                u[a] = 1.0;
                for (int j = l; j >= 0; --j) u = vm(u, R[j]);
                for (int c = 0; c < m; ++c) {
                    HC[2 * (((size_t)b * 64 + q) * G + c)] = u[P->C[c]].real();
                    HC[2 * (((size_t)b * 64 + q) * G + c) + 1] = u[P->C[c]].imag();
                }
            }
        if ((st = dev_upload(P->dgGA, GA.data(), GA.size() * 8)) ||
            (st = dev_upload(P->dgHC, HC.data(), HC.size() * 8)) ||
            (st = dev_upload(P->dgTT, TT.data(), TT.size() * 8)))
            return st;
        g.GA = (const double2 *)P->dgGA.p;
        g.HC = (const double2 *)P->dgHC.p;
        g.TT = (const double2 *)P->dgTT.p;
    }
    P->hkbt = kbt;
    if ((st = dev_upload(P->dgcol, col.data(), col.size())) || (st = dev_upload(P->dgact, act.data(), act.size())) ||
        (st = dev_upload(P->dgpos0, pos0.data(), 128)) || (st = dev_upload(P->dgpos1, pos1.data(), 128)) ||
        (st = dev_upload(P->dgblk, blk.data(), 128)) || (st = dev_upload(P->dgkbt, kbt.data(), 256)) ||
        (st = dev_upload(P->dggpos, gpos.data(), 256)))
        return st;
    g.col = (const uint8_t *)P->dgcol.p;
    g.act = (const uint8_t *)P->dgact.p;
    g.pos0 = (const int8_t *)P->dgpos0.p;
    g.pos1 = (const int8_t *)P->dgpos1.p;
    g.blk = (const int8_t *)P->dgblk.p;
    g.kbt = (const uint16_t *)P->dgkbt.p;
    g.gpos = (const uint16_t *)P->dggpos.p;
    return XF_OK;
}

// Host FP64 precompute of the low-rank factors, uploaded to the device.
xf_status refresh_matrices(xf_plan *P) {
    const int n = P->n, m = P->m, G = P->G, L = P->L;
    std::vector<std::vector<cd>> R(P->n_rot, std::vector<cd>((size_t)n * n));
    for (int l = 0; l < P->n_rot; ++l)
        for (size_t i = 0; i < (size_t)n * n; ++i)
            R[l][i] = cd(P->rot[2 * ((size_t)l * n * n + i)], P->rot[2 * ((size_t)l * n * n + i) + 1]);
    // R'_l = R_l D0_{l-1}: column q of R_l times prod of e^{i theta_j / 2} over
    // the gates j of CPhase layer l-1 that touch mode q.
    P->d0.assign(P->n_rot, std::vector<cd>());
    for (int l = 1; l < P->n_rot; ++l) {
        std::vector<cd> d(n, 1.0);
        for (int j = 0; j < P->k; ++j) {
            if (P->layer[j] != l - 1) continue;
            const cd f = std::polar(1.0, P->theta[j] / 2.0);
            d[P->pairs[2 * j]] *= f;
            d[P->pairs[2 * j + 1]] *= f;
        }
        for (int r = 0; r < n; ++r)
            for (int q = 0; q < n; ++q) R[l][(size_t)r * n + q] *= d[q];
        P->d0[l] = d;
    }
    P->Rp = R;
    std::vector<cd> Phi0((size_t)n * m), Pm, Qm, Tm;
    for (int r = 0; r < n; ++r)
        for (int a = 0; a < m; ++a) Phi0[(size_t)r * m + a] = R[0][(size_t)r * n + P->C[a]];
    P->hPhi0 = Phi0;
    Pm = Phi0;
    if (L >= 1) {
        Qm.assign((size_t)n * m, 0.0);
        matmul(R[1].data(), Phi0.data(), Qm.data(), n, n, m);
        Pm = Qm;
    }
    if (L >= 3) {
        // V(0)[:, C] through every layer (the factors of the positions are
        // formed with the block tables in refresh_gen)
        for (int l = 2; l <= L; ++l) {
            std::vector<cd> X((size_t)n * m, 0.0);
            matmul(R[l].data(), Pm.data(), X.data(), n, n, m);
            Pm = X;
        }
    }
    if (L == 2) {
        Pm.assign((size_t)n * m, 0.0);
        matmul(R[2].data(), Qm.data(), Pm.data(), n, n, m);
        Tm.assign((size_t)n * n, 0.0);
        matmul(R[2].data(), R[1].data(), Tm.data(), n, n, n);
    }
    auto padded = [&](const std::vector<cd> &X) {
        std::vector<double> out((size_t)n * G * 2, 0.0);
        for (int r = 0; r < n; ++r)
            for (int a = 0; a < m; ++a) {
                out[2 * ((size_t)r * G + a)] = X[(size_t)r * m + a].real();
                out[2 * ((size_t)r * G + a) + 1] = X[(size_t)r * m + a].imag();
            }
        return out;
    };
    auto flat = [&](const std::vector<cd> &X) {
        std::vector<double> out(X.size() * 2);
        for (size_t i = 0; i < X.size(); ++i) out[2 * i] = X[i].real(), out[2 * i + 1] = X[i].imag();
        return out;
    };
    auto tofloat = [](const std::vector<double> &x) {
        std::vector<float> f(x.size());
        for (size_t i = 0; i < x.size(); ++i) f[i] = (float)x[i];
        return f;
    };
    xf_status st;
    auto up = [&](DevBuf &b, const std::vector<double> &h) { return dev_upload(b, h.data(), h.size() * 8); };
    auto upf = [&](DevBuf &b, const std::vector<double> &h) {
        const std::vector<float> f = tofloat(h);
        return dev_upload(b, f.data(), f.size() * 4);
    };
    const std::vector<double> hP = padded(Pm), hPhi = padded(Phi0);
    if ((st = up(P->dP, hP)) || (st = up(P->dPhi0, hPhi)) || (st = upf(P->fPhi0, hPhi))) return st;
    if (L == 1) {
        const std::vector<double> a1 = flat(R[1]);
        if ((st = up(P->dA1, a1)) || (st = upf(P->fA1, a1))) return st;
    } else if (L == 2) {
        const std::vector<double> a1 = flat(Tm), a2 = flat(R[2]), r1 = flat(R[1]), q = padded(Qm);
        if ((st = up(P->dA1, a1)) || (st = upf(P->fA1, a1)) || (st = up(P->dA2, a2)) ||
            (st = upf(P->fA2, a2)) || (st = up(P->dR1, r1)) || (st = upf(P->fR1, r1)) ||
            (st = up(P->dQ, q)) || (st = upf(P->fQ, q)))
            return st;
    }
    P->nxterms = -1;
    return refresh_gen(P);
}

xf_status refresh_table(xf_plan *P) {
    const std::vector<uint32_t> T = sampling_table(P->theta);
    return dev_upload(P->dT, T.data(), T.size() * 4);
}

// Exact mode: all 2^k trajectories grouped by key, weights summed in
// ascending x (Sec. III-B Eq. 8-9).  Without derivatives, keys whose weight
// sums to exactly zero are dropped.  With derivatives (for the backward
// pass), dw[key][j] = sum over its x of dw(x)/dtheta_j is stored as well and
// keys are kept while any of weight or derivatives is non-zero.
// Exact mode: the prefix tree of the term list over its flipped positions
// (lemma_tree.h), for one or more CPhase layers under the general lemma.  Tree positions are the (block, position) pairs some term flips, in
// an order chosen to minimise the anchors; a pattern's anchor chain is the
// prefixes of 4, 8, ... of its positions (in that order) that leave it 1 to 4
// more; each anchor keeps the positions beyond its own that its descendants
// use.  No tree (has_tree = false) where more than kTreeMaxM positions are
// flipped in all.
xf_status build_tree(xf_plan *P, const std::vector<uint64_t> &keys, const std::vector<double> &w) {
    P->has_tree = false;
    const xf::GenPlan &g = P->gen;
    if (g.nblk == 0 || P->L < 1 || keys.empty() || P->hkbt.size() < 128) return XF_OK;
    // the keys' flipped positions per block (a key bit flips one or two positions)
    std::vector<uint32_t> code_of(2 * 256, 0xFFFFFFFFu);
    std::vector<uint16_t> codes;
    std::vector<std::vector<uint16_t>> kpos(keys.size());
    for (size_t i = 0; i < keys.size(); ++i) {
        uint64_t pm[2] = {0, 0};
        for (uint64_t key = keys[i]; key; key &= key - 1) {
            const int j = __builtin_ctzll(key);
            for (int e = 0; e < 2; ++e) {
                const uint16_t v = P->hkbt[2 * j + e];
                if (v != 0xFFFF) pm[v >> 8] ^= 1ull << (v & 0xFF);
            }
        }
        for (int b = 0; b < 2; ++b)
            for (uint64_t mm = pm[b]; mm; mm &= mm - 1) {
                const uint16_t c = (uint16_t)((b << 8) | __builtin_ctzll(mm));
                kpos[i].push_back(c);
                codes.push_back(c);
            }
    }
    std::sort(codes.begin(), codes.end());
    codes.erase(std::unique(codes.begin(), codes.end()), codes.end());
    const int M = (int)codes.size();
    if (M == 0 || M > xf::kTreeMaxM) return XF_OK;
    for (int t = 0; t < M; ++t) code_of[codes[t]] = (uint32_t)t;
    // distinct tree masks with summed weights
    std::vector<std::pair<uint32_t, cd>> pats;
    {
        std::vector<std::pair<uint32_t, cd>> all(keys.size());
        for (size_t i = 0; i < keys.size(); ++i) {
            uint32_t m = 0;
            for (uint16_t c : kpos[i]) m |= 1u << code_of[c];
            all[i] = {m, cd(w[2 * i], w[2 * i + 1])};
        }
        std::sort(all.begin(), all.end(), [](const std::pair<uint32_t, cd> &a, const std::pair<uint32_t, cd> &b) {
            return a.first < b.first;
        });
        for (size_t i = 0; i < all.size();) {
            size_t e = i;
            cd acc = 0.0;
            while (e < all.size() && all[e].first == all[i].first) acc += all[e++].second;
            if (acc != 0.0) pats.emplace_back(all[i].first, acc);
            i = e;
        }
    }
    // The order of the positions decides how many prefixes the patterns
    // share (how many anchors the tree has): the natural order, the gates'
    // order and seeded random orders of the gates and of the positions are
    // tried, the best is improved by swapping pairs of positions while that
    // does not add anchors, and the order with the fewest anchors is kept
    // (deterministic for a given plan; reused while the set of patterns is
    // unchanged).
    uint64_t pkey = 1469598103934665603ull ^ (uint64_t)M;
    for (const auto &pw : pats) pkey = (pkey ^ pw.first) * 1099511628211ull;
    for (uint16_t c : codes) pkey = (pkey ^ c) * 1099511628211ull;
    if (pkey == P->tree_key && P->tree_codes.size() == (size_t)M) {
        std::vector<int> rank_of(M);
        for (int r = 0; r < M; ++r) rank_of[code_of[P->tree_codes[r]]] = r;
        for (auto &pw : pats) {
            uint32_t rm = 0;
            for (uint32_t m = pw.first; m; m &= m - 1) rm |= 1u << rank_of[__builtin_ctz(m)];
            pw.first = rm;
        }
        codes = P->tree_codes;
        std::sort(pats.begin(), pats.end(), [](const std::pair<uint32_t, cd> &a, const std::pair<uint32_t, cd> &b) {
            return a.first < b.first;
        });
    } else {
        std::vector<std::vector<int>> gate_pos;
        for (int j = 0; j < P->k && j < 64; ++j) {
            std::vector<int> v;
            for (uint64_t gk = P->gkey[j]; gk; gk &= gk - 1) {
                const int b = __builtin_ctzll(gk);
                for (int e = 0; e < 2 && b < 64; ++e) {
                    const uint16_t c = P->hkbt[2 * b + e];
                    if (c != 0xFFFF && code_of[c] != 0xFFFFFFFFu) v.push_back((int)code_of[c]);
                }
            }
            gate_pos.push_back(v);
        }
        auto from_gates = [&](const std::vector<int> &gorder) {
            std::vector<int> ord;
            std::vector<char> in(M, 0);
            for (int j : gorder)
                for (int t : gate_pos[j])
                    if (!in[t]) in[t] = 1, ord.push_back(t);
            for (int t = 0; t < M; ++t)
                if (!in[t]) ord.push_back(t);
            return ord;
        };
        // anchors of an order (ord[r] = the position taking rank r)
        std::vector<uint32_t> seen;
        auto anchors_of = [&](const std::vector<int> &ord) {
            int rank[xf::kTreeMaxM];
            for (int r = 0; r < M; ++r) rank[ord[r]] = r;
            seen.clear();
            for (const auto &pw : pats) {
                uint32_t rm = 0;
                for (uint32_t m = pw.first; m; m &= m - 1) rm |= 1u << rank[__builtin_ctz(m)];
                // the prefixes of 4, 8, ... positions (ascending rank) short of the whole pattern
                const int r = __builtin_popcount(rm);
                uint32_t pre = 0;
                int cnt = 0;
                for (uint32_t m = rm; m; m &= m - 1) {
                    pre |= m & (~m + 1);
                    if (++cnt % 4 == 0) {
                        if (cnt >= r) break;
                        seen.push_back(pre);
                    }
                }
            }
            std::sort(seen.begin(), seen.end());
            return (size_t)(std::unique(seen.begin(), seen.end()) - seen.begin());
        };
        std::vector<int> best(M);
        for (int t = 0; t < M; ++t) best[t] = t;
        size_t best_n = anchors_of(best);
        std::vector<int> gorder(gate_pos.size());
        for (size_t j = 0; j < gorder.size(); ++j) gorder[j] = (int)j;
        auto consider = [&](const std::vector<int> &ord) {
            const size_t n = anchors_of(ord);
            if (n < best_n) best_n = n, best = ord;
        };
        consider(from_gates(gorder));
        uint64_t z = 0x9E3779B97F4A7C15ull;   // splitmix64, fixed seed
        auto next = [&]() {
            uint64_t x = (z += 0x9E3779B97F4A7C15ull);
            x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
            x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
            return x ^ (x >> 31);
        };
        const size_t work = pats.size() * (size_t)M;
        const int tries = work > (8u << 20) ? 4 : (work > (1u << 20) ? 16 : 48);
        for (int it = 0; it < tries; ++it) {
            std::vector<int> g = gorder, o(M);
            for (int i = (int)g.size() - 1; i > 0; --i) std::swap(g[i], g[next() % (uint64_t)(i + 1)]);
            consider(from_gates(g));
            for (int t = 0; t < M; ++t) o[t] = t;
            for (int i = M - 1; i > 0; --i) std::swap(o[i], o[next() % (uint64_t)(i + 1)]);
            consider(o);
        }
        // pairwise swaps, kept unless they add anchors (about 6e7 position
        // visits in all)
        const int swaps = (int)std::min<size_t>(600, (60u << 20) / std::max<size_t>(work, 1));
        for (int it = 0; it < swaps && M > 1; ++it) {
            std::vector<int> o = best;
            const int a = (int)(next() % (uint64_t)M), b = (int)(next() % (uint64_t)M);
            if (a == b) continue;
            std::swap(o[a], o[b]);
            const size_t n = anchors_of(o);
            if (n <= best_n) best_n = n, best = o;
        }
        int rank[xf::kTreeMaxM];
        for (int r = 0; r < M; ++r) rank[best[r]] = r;
        std::vector<uint16_t> c2(M);
        for (int r = 0; r < M; ++r) c2[r] = codes[best[r]];
        codes = c2;
        for (auto &pw : pats) {
            uint32_t rm = 0;
            for (uint32_t m = pw.first; m; m &= m - 1) rm |= 1u << rank[__builtin_ctz(m)];
            pw.first = rm;
        }
        std::sort(pats.begin(), pats.end(), [](const std::pair<uint32_t, cd> &a, const std::pair<uint32_t, cd> &b) {
            return a.first < b.first;
        });
        P->tree_key = pkey;
        P->tree_codes = codes;
    }
    struct Anc {
        int level = 0, parent = -1;
        int j[4] = {0, 0, 0, 0};
        uint32_t need = 0;   // positions beyond its own that its descendants use
        std::vector<int> kids, pats;
        bool pair_first = false;   // a leaf taken together with the next sibling leaf
    };
    std::vector<Anc> an(1);
    std::vector<std::pair<uint32_t, int>> ids;   // prefix mask -> anchor, sorted on insertion
    auto find_anchor = [&](uint32_t m) -> int {
        auto it = std::lower_bound(ids.begin(), ids.end(), std::make_pair(m, -1));
        return (it != ids.end() && it->first == m) ? it->second : -1;
    };
    for (size_t pi = 0; pi < pats.size(); ++pi) {
        int bits[32];
        int r = 0;
        for (uint32_t m = pats[pi].first; m; m &= m - 1) bits[r++] = __builtin_ctz(m);
        const int q = r > 0 ? (r - 1) / 4 : 0;
        int chain[9] = {0};
        uint32_t pre = 0;
        for (int lv = 1; lv <= q; ++lv) {
            for (int u = 4 * lv - 4; u < 4 * lv; ++u) pre |= 1u << bits[u];
            int id = find_anchor(pre);
            if (id < 0) {
                id = (int)an.size();
                Anc a;
                a.level = lv;
                a.parent = chain[lv - 1];
                for (int u = 0; u < 4; ++u) a.j[u] = bits[4 * lv - 4 + u];
                an.push_back(a);
                an[chain[lv - 1]].kids.push_back(id);
                ids.insert(std::lower_bound(ids.begin(), ids.end(), std::make_pair(pre, -1)), std::make_pair(pre, id));
            }
            chain[lv] = id;
        }
        for (int lv = 0; lv <= q; ++lv) {
            const int last = lv == 0 ? -1 : an[chain[lv]].j[3];
            for (int u = 0; u < r; ++u)
                if (bits[u] > last) an[chain[lv]].need |= 1u << bits[u];
        }
        an[chain[q]].pats.push_back((int)pi);
    }
    // the positions each anchor keeps: the root all M, others their need
    auto rlist = [&](int a) {
        std::vector<int> v;
        if (a == 0) {
            for (int t = 0; t < M; ++t) v.push_back(t);
        } else {
            for (uint32_t m = an[a].need; m; m &= m - 1) v.push_back(__builtin_ctz(m));
        }
        return v;
    };
    auto index_in = [](const std::vector<int> &v, int x) {
        return (int)(std::lower_bound(v.begin(), v.end(), x) - v.begin());
    };
    std::vector<xf::TreeAnchor> tanc;
    std::vector<uint8_t> tridx;
    std::vector<xf::TreePat> tpat;
    int maxnr[xf::kTreeLevels] = {M, 0, 0, 0, 0, 0, 0, 0};
    int maxr = 1;
    auto emit_pats = [&](int a, const std::vector<int> &R) {
        const int last = a == 0 ? -1 : an[a].j[3];
        for (int pi : an[a].pats) {
            xf::TreePat tp{};
            tp.w.x = pats[pi].second.real();
            tp.w.y = pats[pi].second.imag();
            tp.level = (uint8_t)an[a].level;
            int r = 0;
            for (uint32_t m = pats[pi].first; m; m &= m - 1) {
                const int b = __builtin_ctz(m);
                if (b > last) tp.idx[r++] = (uint8_t)index_in(R, b);
            }
            tp.r = (uint8_t)r;
            tpat.push_back(tp);
        }
    };
    emit_pats(0, rlist(0));
    const int nroot = (int)tpat.size();
    // leaves (anchors without children) first among their siblings, in
    // pairs where two follow each other
    for (Anc &a : an) {
        std::stable_partition(a.kids.begin(), a.kids.end(), [&](int c) { return an[c].kids.empty(); });
        size_t nl = 0;
        while (nl < a.kids.size() && an[a.kids[nl]].kids.empty()) ++nl;
        for (size_t k = 0; k + 1 < nl; k += 2) an[a.kids[k]].pair_first = true;
    }
    // depth-first over the anchors (iterative; children in that order);
    // each emitted anchor's parent (emitted index, -1 for the root)
    std::vector<int> emit_of(an.size(), -1), parent_of;
    std::vector<std::pair<int, size_t>> stack;
    stack.emplace_back(0, 0);
    while (!stack.empty()) {
        const int a = stack.back().first;
        const size_t k = stack.back().second;
        if (k >= an[a].kids.size()) {
            stack.pop_back();
            continue;
        }
        ++stack.back().second;
        const int c = an[a].kids[k];
        const std::vector<int> RP = rlist(a), RC = rlist(c);
        xf::TreeAnchor ta{};
        ta.level = (uint8_t)an[c].level;
        ta.nr = (uint8_t)RC.size();
        ta.pnr = (uint8_t)RP.size();
        for (int u = 0; u < 4; ++u) ta.j[u] = (uint8_t)index_in(RP, an[c].j[u]);
        ta.roff = (uint32_t)tridx.size();
        for (int x : RC) tridx.push_back((uint8_t)index_in(RP, x));
        ta.pat0 = (uint32_t)tpat.size();
        emit_pats(c, RC);
        ta.npat = (uint32_t)(tpat.size() - ta.pat0);
        const bool leaf = an[c].kids.empty();
        ta.pad = (uint8_t)((leaf ? 1 : 0) | (an[c].pair_first ? 2 : 0));
        emit_of[c] = (int)tanc.size();
        parent_of.push_back(a == 0 ? -1 : emit_of[a]);
        tanc.push_back(ta);
        // a leaf keeps no matrix of its own: the levels' slots hold the others
        if (!leaf) maxnr[ta.level] = std::max(maxnr[ta.level], (int)ta.nr);
        maxr = std::max(maxr, (int)ta.nr);
        stack.emplace_back(c, 0);
    }
    // parts of the walk for small batches: up to 1024 runs of the
    // depth-first order (never between the two leaves of a pair), cut where
    // the estimated work (per anchor a block elimination, its matrix and its
    // patterns' passes) reaches equal shares; a part starts by recomputing
    // the matrices of its first anchor's ancestors (any run is then
    // self-contained: an anchor's parent precedes it, in the run or among
    // those ancestors)
    std::vector<uint32_t> pstart(1, 0);
    {
        std::vector<double> pre(tanc.size() + 1, 0.0);
        for (size_t x = 0; x < tanc.size(); ++x) {
            const double nr = tanc[x].nr;
            pre[x + 1] = pre[x] + 4.0 + std::ceil(nr * nr / 64.0) + std::ceil(tanc[x].npat / 4.0);
        }
        std::vector<size_t> cuts;
        for (size_t x = 1; x < tanc.size(); ++x)
            if (!(tanc[x - 1].pad & 2)) cuts.push_back(x);
        const int want = (int)std::min<size_t>(1024, cuts.size() + 1);
        size_t c = 0;
        for (int kq = 1; kq < want; ++kq) {
            const double target = pre.back() * kq / want;
            while (c < cuts.size() && (pre[cuts[c]] < target || cuts[c] <= pstart.back())) ++c;
            if (c >= cuts.size()) break;
            pstart.push_back((uint32_t)cuts[c]);
        }
        pstart.push_back((uint32_t)tanc.size());
    }
    std::vector<uint32_t> pchain((pstart.size() - 1) * 8, 0xFFFFFFFFu);
    for (size_t q = 0; q + 1 < pstart.size(); ++q) {
        if (pstart[q] >= tanc.size()) continue;
        for (int y = parent_of[pstart[q]]; y >= 0; y = parent_of[y]) pchain[q * 8 + tanc[y].level] = (uint32_t)y;
    }
    xf::DevTree &t = P->tree;
    t = xf::DevTree{};
    t.nparts = (int)pstart.size() - 1;
    t.nanc = (int)tanc.size();
    t.nroot = nroot;
    t.npat = (int)tpat.size();
    t.M = M;
    int off = 0;
    for (int l = 0; l < xf::kTreeLevels; ++l) {
        t.slot[l] = off;
        off += maxnr[l] * maxnr[l];
    }
    t.maxr = maxr;
    t.toff = off;
    t.doff = off + 8 * maxr;                  // two T buffers (a pair of leaves)
    t.soff = t.doff + xf::kTreeLevels + 2;    // the levels' prefix dets, then the pair's
    t.lds = 16 * (t.soff + 17 * xf::kTreeStage);
    t.growth2 = P->tree_growth * P->tree_growth;
    if (t.lds > 64 * 1024) return XF_OK;
    // every index the kernel follows stays inside its matrix
    for (const xf::TreeAnchor &a : tanc) {
        if (a.level < 1 || a.level >= xf::kTreeLevels || a.pnr > maxnr[a.level - 1] || a.nr > maxr ||
            (!(a.pad & 1) && a.nr > maxnr[a.level]) || ((a.pad & 2) && (&a == &tanc.back() || !((&a)[1].pad & 1) ||
                                                                        (&a)[1].level != a.level || (&a)[1].pnr != a.pnr)))
            return fail(XF_EDEVICE, "internal error: prefix tree anchor size");
        for (int u = 0; u < 4; ++u)
            if (a.j[u] >= a.pnr) return fail(XF_EDEVICE, "internal error: prefix tree anchor index");
        for (int x = 0; x < a.nr; ++x)
            if (tridx[a.roff + x] >= a.pnr) return fail(XF_EDEVICE, "internal error: prefix tree row index");
        for (uint32_t q = a.pat0; q < a.pat0 + a.npat; ++q)
            for (int u = 0; u < tpat[q].r; ++u)
                if (tpat[q].r > 4 || tpat[q].idx[u] >= a.nr)
                    return fail(XF_EDEVICE, "internal error: prefix tree pattern index");
    }
    for (size_t q = 0; q + 1 < pstart.size(); ++q) {
        if (pstart[q] >= tanc.size()) continue;
        for (int l = 1; l < tanc[pstart[q]].level; ++l)
            if (pchain[q * 8 + l] >= tanc.size() || tanc[pchain[q * 8 + l]].level != l || (tanc[pchain[q * 8 + l]].pad & 1))
                return fail(XF_EDEVICE, "internal error: prefix tree part ancestors");
    }
    for (int q = 0; q < nroot; ++q)
        for (int u = 0; u < tpat[q].r; ++u)
            if (tpat[q].r > 4 || tpat[q].idx[u] >= M) return fail(XF_EDEVICE, "internal error: prefix tree root index");
    xf_status st;
    // the kernel's prefetches read, unconditionally, one element past an
    // anchor's R indices or patterns when it has none, and element 0 of the
    // anchors: one element of padding each
    tridx.push_back(0);
    tpat.push_back(xf::TreePat{});
    if (tanc.empty()) tanc.push_back(xf::TreeAnchor{});
    if ((st = dev_upload(P->dtanc, tanc.data(), tanc.size() * sizeof(xf::TreeAnchor))) ||
        (st = dev_upload(P->dtridx, tridx.data(), tridx.size())) ||
        (st = dev_upload(P->dtpat, tpat.data(), tpat.size() * sizeof(xf::TreePat))) ||
        (st = dev_upload(P->dtrpos, codes.data(), codes.size() * sizeof(uint16_t))) ||
        (st = dev_upload(P->dtpart, pstart.data(), pstart.size() * sizeof(uint32_t))) ||
        (st = dev_upload(P->dtchain, pchain.data(), pchain.size() * sizeof(uint32_t))))
        return st;
    t.anc = (const xf::TreeAnchor *)P->dtanc.p;
    t.ridx = (const uint8_t *)P->dtridx.p;
    t.pat = (const xf::TreePat *)P->dtpat.p;
    t.rpos = (const uint16_t *)P->dtrpos.p;
    t.pstart = (const uint32_t *)P->dtpart.p;
    t.pchain = (const uint32_t *)P->dtchain.p;
    P->has_tree = true;
    return XF_OK;
}

xf_status build_exact_terms(xf_plan *P, bool with_dw) {
    const int k = P->k;
    const uint64_t nx = 1ull << k;
    std::vector<cd> f0(k), f1(k);
    for (int j = 0; j < k; ++j) {
        f0[j] = cd(std::cos(P->theta[j] / 4.0), 0.0);
        f1[j] = cd(0.0, std::sin(P->theta[j] / 4.0));
    }
    std::vector<std::pair<uint64_t, uint64_t>> kx;
    kx.reserve(nx);
    for (uint64_t x = 0; x < nx; ++x) {
        uint64_t key = 0;
        for (int j = 0; j < k; ++j)
            if ((x >> j) & 1) key ^= P->gkey[j];
        kx.emplace_back(key, x);
    }
    std::sort(kx.begin(), kx.end());
    // d/dtheta of cos(theta/4) and of i sin(theta/4)
    std::vector<cd> g0(k), g1(k);
    for (int j = 0; j < k; ++j) {
        g0[j] = cd(-std::sin(P->theta[j] / 4.0) / 4.0, 0.0);
        g1[j] = cd(0.0, std::cos(P->theta[j] / 4.0) / 4.0);
    }
    std::vector<uint64_t> keys;
    std::vector<double> w, dw;
    std::vector<cd> dacc(k), fac(k);
    for (size_t i = 0; i < kx.size();) {
        size_t e = i;
        cd acc = 0.0;
        std::fill(dacc.begin(), dacc.end(), cd(0.0));
        while (e < kx.size() && kx[e].first == kx[i].first) {
            const uint64_t x = kx[e].second;
            cd wx = 1.0;
            for (int j = 0; j < k; ++j) {
                fac[j] = ((x >> j) & 1) ? f1[j] : f0[j];
                wx *= fac[j];
            }
            acc += wx;
            if (with_dw) {
                for (int j = 0; j < k; ++j) {
                    cd d = ((x >> j) & 1) ? g1[j] : g0[j];
                    for (int i2 = 0; i2 < k; ++i2)
                        if (i2 != j) d *= fac[i2];
                    dacc[j] += d;
                }
            }
            ++e;
        }
        bool keep = acc != 0.0;
        for (int j = 0; j < k && with_dw && !keep; ++j) keep = dacc[j] != 0.0;
        if (keep) {
            keys.push_back(kx[i].first);
            w.push_back(acc.real());
            w.push_back(acc.imag());
            if (with_dw)
                for (int j = 0; j < k; ++j) dw.push_back(dacc[j].real()), dw.push_back(dacc[j].imag());
        }
        i = e;
    }
    xf_status st;
    if ((st = dev_upload(P->dxkeys, keys.data(), keys.size() * 8)) ||
        (st = dev_upload(P->dxw, w.data(), w.size() * 8)))
        return st;
    if (with_dw && (st = dev_upload(P->dxdw, dw.data(), dw.size() * 8))) return st;
    P->nxterms = (int64_t)keys.size();
    P->xterms_have_dw = with_dw;
    return build_tree(P, keys, w);
}

xf::DevPlan snapshot(const xf_plan *P) {
    xf::DevPlan d{};
    d.n = P->n, d.m = P->m, d.L = P->L, d.k = P->k, d.G = P->G;
    d.keykind = P->keykind, d.keybits = P->keybits, d.off1 = P->off1;
    d.P = (const double2 *)P->dP.p;
    d.Phi0 = (const double2 *)P->dPhi0.p;
    d.A1 = (const double2 *)P->dA1.p;
    d.A2 = (const double2 *)P->dA2.p;
    d.Q = (const double2 *)P->dQ.p;
    d.R1 = (const double2 *)P->dR1.p;
    d.fPhi0 = (const float2 *)P->fPhi0.p;
    d.fA1 = (const float2 *)P->fA1.p;
    d.fA2 = (const float2 *)P->fA2.p;
    d.fQ = (const float2 *)P->fQ.p;
    d.fR1 = (const float2 *)P->fR1.p;
    d.keymode = (const uint8_t *)P->dkeymode.p;
    d.T = (const uint32_t *)P->dT.p;
    d.gkey = (const uint64_t *)P->dgkey.p;
    d.gmode = (const uint64_t *)P->dgmode.p;
    d.glayer = (const int32_t *)P->dglayer.p;
    d.gneg = (const uint8_t *)P->dgneg.p;
    d.scale = 1.0;
    d.mixed_cond = P->mixed_cond;
    return d;
}

void plan_free(xf_plan *P) {
    for (DevBuf *b : {&P->dP, &P->dPhi0, &P->dA1, &P->dA2, &P->dQ, &P->dR1, &P->fPhi0, &P->fA1,
                      &P->fA2, &P->fQ, &P->fR1, &P->dkeymode, &P->dT, &P->dgkey, &P->dgmode,
                      &P->dglayer, &P->dgneg, &P->dnterm, &P->dxkeys, &P->dxw, &P->dxdw, &P->dpart,
                      &P->dgsum, &P->dekey, &P->decnt, &P->decount, &P->dgcol, &P->dgact, &P->dgpos0,
                      &P->dgpos1, &P->dgblk, &P->dgkbt, &P->dggpos, &P->dflags, &P->dgGA, &P->dgHC, &P->dgTT, &P->dgsetup,
                      &P->dtanc, &P->dtridx, &P->dtpat, &P->dtrpos, &P->dtpart, &P->dtchain})
        dev_free(*b);
    for (hipEvent_t e : P->ev) (void)hipEventDestroy(e);
    P->ev.clear();
    P->nev = 0;
}

// At least n timing events.
xf_status ensure_events(xf_plan *P, size_t n) {
    while (P->ev.size() < n) {
        hipEvent_t e;
        if (hipEventCreate(&e) != hipSuccess) return fail(XF_EDEVICE, "hipEventCreate failed");
        P->ev.push_back(e);
    }
    return ok();
}



// Workspace of the determinant-lemma kernels for chunks of `chunk` bitstrings
// with `cap` entries each (grown on demand; synchronises s before a resize).
xf_status ensure_lemma_workspace(xf_plan *P, int64_t chunk, uint64_t cap, hipStream_t s) {
    if (P->dekey.bytes >= (size_t)chunk * cap * 8 && P->decnt.bytes >= (size_t)chunk * cap * 8 &&
        P->decount.bytes >= (size_t)chunk * 4)
        return XF_OK;
    if (hipStreamSynchronize(s) != hipSuccess) return fail(XF_EDEVICE, "stream synchronisation failed");
    xf_status st;
    if ((st = dev_upload(P->dekey, nullptr, (size_t)chunk * cap * 8)) ||
        (st = dev_upload(P->decnt, nullptr, (size_t)chunk * cap * 8)) ||
        (st = dev_upload(P->decount, nullptr, (size_t)chunk * 4)))
        return st;
    return XF_OK;
}

xf_status set_gate_tables(xf_plan *P) {
    // signs of the angles (phase i or -i of a d_1 choice)
    P->gneg.assign(std::max(P->k, 1), 0);
    for (int j = 0; j < P->k; ++j) P->gneg[j] = P->theta[j] < 0.0 ? 1 : 0;
    return dev_upload(P->dgneg, P->gneg.data(), P->gneg.size());
}

}  // namespace

extern "C" {

const char *xf_last_error(void) { return g_err.c_str(); }

xf_status xf_plan_create(const xf_circuit *c, xf_bits128 input, xf_precision precision, int device,
                         xf_plan **plan) {
    if (!plan) return fail(XF_EINVAL, "plan output pointer is NULL");
    *plan = nullptr;
    if (!c) return fail(XF_EINVAL, "circuit is NULL");
    if (c->n < 1) return fail(XF_EINVAL, "n must be >= 1");
    if (c->n > 128) return fail(XF_EUNSUPPORTED, "n = %d > 128", c->n);
    if (c->n_rot < 1) return fail(XF_EINVAL, "n_rot must be >= 1");
    if (c->n_rot > kMaxRot) return fail(XF_EUNSUPPORTED, "n_rot = %d > %d", c->n_rot, kMaxRot);
    if (c->n_rot > 3 && c->k > 63)
        return fail(XF_EUNSUPPORTED, "more than two CPhase layers need k <= 63 (k = %d)", c->k);
    if (!c->rot) return fail(XF_EINVAL, "rot is NULL");
    if (c->k < 0) return fail(XF_EINVAL, "k must be >= 0");
    if (c->k > 0 && (!c->pairs || !c->layer || !c->theta)) return fail(XF_EINVAL, "pairs/layer/theta is NULL");
    if (precision != XF_FP64 && precision != XF_MIXED) return fail(XF_EINVAL, "unknown precision");
    const int n = c->n, k = c->k, n_rot = c->n_rot;
    for (int j = 0; j < k; ++j) {
        const int a = c->pairs[2 * j], b = c->pairs[2 * j + 1];
        if (a < 0 || a >= n || b < 0 || b >= n || a == b) return fail(XF_EINVAL, "gate %d has invalid pair (%d, %d)", j, a, b);
        if (c->layer[j] < 0 || c->layer[j] > n_rot - 2) return fail(XF_EINVAL, "gate %d has invalid layer %d", j, c->layer[j]);
    }
    if (n < 128) {
        const uint64_t hi0 = n >= 64 ? 0ull : (~0ull << n);
        const uint64_t hi1 = n <= 64 ? ~0ull : (~0ull << (n - 64));
        if ((input.w[0] & hi0) || (input.w[1] & hi1)) return fail(XF_EINVAL, "input has bits at or above n");
    }
    const int m = __builtin_popcountll(input.w[0]) + __builtin_popcountll(input.w[1]);
    if (m > 64) return fail(XF_EUNSUPPORTED, "eta = %d > 64", m);
    xf_status st = check_params(n, n_rot, c->rot, k, c->theta);
    if (st) return st;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev)
        return fail(XF_EDEVICE, "device %d not available", device);

    xf_plan *P = new (std::nothrow) xf_plan();
    if (!P) return fail(XF_ENOMEM, "host allocation failed");
    P->device = device;
    P->n = n, P->n_rot = n_rot, P->k = k, P->m = m, P->L = n_rot - 1;
    P->precision = precision;
    P->G = 4;
    while (P->G < m) P->G *= 2;
    P->rot.assign(c->rot, c->rot + (size_t)n_rot * n * n * 2);
    P->pairs.assign(c->pairs ? c->pairs : nullptr, c->pairs ? c->pairs + 2 * k : nullptr);
    P->layer.assign(c->layer ? c->layer : nullptr, c->layer ? c->layer + k : nullptr);
    P->theta.assign(c->theta ? c->theta : nullptr, c->theta ? c->theta + k : nullptr);
    for (int q = 0; q < n; ++q)
        if ((input.w[q >> 6] >> (q & 63)) & 1) P->C.push_back(q);

    // Flip-pattern keys: the modes touched by each CPhase layer, packed (one
    // or two layers), or the trajectory itself.
    std::vector<std::vector<int>> act(std::max(2, n_rot - 1));
    for (int j = 0; j < k; ++j)
        for (int side = 0; side < 2; ++side) act[P->layer[j]].push_back(P->pairs[2 * j + side]);
    for (auto &v : act) {
        std::sort(v.begin(), v.end());
        v.erase(std::unique(v.begin(), v.end()), v.end());
    }
    P->off1 = (int)act[0].size();
    P->keybits = (int)(act[0].size() + act[1].size());
    P->keymode.assign(64, 0);
    P->gkey.assign(std::max(k, 1), 0);
    P->gmode.assign(2 * std::max(k, 1), 0);
    std::vector<int32_t> glayer(std::max(k, 1), 0);
    if (P->keybits <= 63 && n_rot <= 3) P->keykind = 0;
    else if (k <= 63) P->keykind = 1;
    else P->keykind = -1;
    for (size_t i = 0; i < act[0].size() && P->keykind == 0; ++i) P->keymode[i] = (uint8_t)act[0][i];
    for (size_t i = 0; i < act[1].size() && P->keykind == 0; ++i) P->keymode[P->off1 + i] = (uint8_t)act[1][i];
    for (int j = 0; j < k; ++j) {
        const int l = P->layer[j];
        glayer[j] = l;
        for (int side = 0; side < 2; ++side) {
            const int q = P->pairs[2 * j + side];
            P->gmode[2 * j + (q >> 6)] ^= 1ull << (q & 63);
            if (P->keykind == 0) {
                const int pos = (l == 0 ? 0 : P->off1) +
                                (int)(std::lower_bound(act[l].begin(), act[l].end(), q) - act[l].begin());
                P->gkey[j] ^= 1ull << pos;
            }
        }
        if (P->keykind == 1) P->gkey[j] = 1ull << j;
    }

    DeviceGuard guard(device);
    if (!guard.okay) {
        delete P;
        return fail(XF_EDEVICE, "hipSetDevice(%d) failed", device);
    }
    if (xf::prepare_kernels(P->G) != hipSuccess) {
        delete P;
        return fail(XF_EDEVICE, "could not configure kernels");
    }
    if ((st = dev_upload(P->dkeymode, P->keymode.data(), 64)) ||
        (st = dev_upload(P->dgkey, P->gkey.data(), P->gkey.size() * 8)) ||
        (st = dev_upload(P->dgmode, P->gmode.data(), P->gmode.size() * 8)) ||
        (st = dev_upload(P->dglayer, glayer.data(), glayer.size() * 4)) ||
        (st = set_gate_tables(P)) || (st = dev_upload(P->dnterm, nullptr, 64)) ||
        (st = refresh_matrices(P)) || (st = refresh_table(P))) {
        plan_free(P);
        delete P;
        return st;
    }
    if (hipMemset(P->dnterm.p, 0, 64) != hipSuccess) {
        plan_free(P);
        delete P;
        return fail(XF_EDEVICE, "hipMemset failed");
    }
    *plan = P;
    return ok();
}

xf_status xf_plan_set_params(xf_plan *P, const double *rot, const double *theta) {
    if (!plan_valid(P)) return fail(XF_EINVAL, "invalid plan");
    P->fwd_valid = false;
    const double *r = rot ? rot : P->rot.data();
    const double *th = theta ? theta : P->theta.data();
    xf_status st = check_params(P->n, P->n_rot, r, P->k, th);
    if (st) return st;
    if (rot) P->rot.assign(rot, rot + P->rot.size());
    if (theta) P->theta.assign(theta, theta + P->k);
    DeviceGuard guard(P->device);
    if (!guard.okay) return fail(XF_EDEVICE, "hipSetDevice failed");
    if (hipDeviceSynchronize() != hipSuccess) return fail(XF_EDEVICE, "device synchronisation failed");
    if ((st = refresh_matrices(P)) || (st = set_gate_tables(P))) return st;
    return ok();
}

xf_status xf_plan_refreeze(xf_plan *P) {
    if (!plan_valid(P)) return fail(XF_EINVAL, "invalid plan");
    P->fwd_valid = false;
    DeviceGuard guard(P->device);
    if (!guard.okay) return fail(XF_EDEVICE, "hipSetDevice failed");
    if (hipDeviceSynchronize() != hipSuccess) return fail(XF_EDEVICE, "device synchronisation failed");
    xf_status st;
    if ((st = refresh_table(P)) || (st = set_gate_tables(P))) return st;
    return ok();
}

xf_status xf_plan_destroy(xf_plan *P) {
    if (!P) return ok();
    {
        DeviceGuard guard(P->device);
        hipDeviceSynchronize();
        plan_free(P);
    }
    delete P;
    return ok();
}

xf_status xf_extent(const xf_plan *P, double *xi) {
    if (!plan_valid(P) || !xi) return fail(XF_EINVAL, "invalid plan or NULL output");
    *xi = extent_of(P->theta);
    return ok();
}

xf_status xf_trajectory_bound(double eps, double delta, double p_max, double xi, int64_t *t) {
    if (!t) return fail(XF_EINVAL, "NULL output");
    if (!(eps > 0.0) || !(delta > 0.0 && delta < 1.0) || !(p_max >= 0.0 && p_max <= 1.0) || !(xi >= 1.0) ||
        !std::isfinite(eps) || !std::isfinite(xi))
        return fail(XF_EINVAL, "need eps > 0, 0 < delta < 1, 0 <= p_max <= 1, xi >= 1");
    const double num = (std::sqrt(xi) + std::sqrt(p_max)) * (std::sqrt(xi) + std::sqrt(p_max));
    const double gap = std::sqrt(p_max + eps) - std::sqrt(p_max);
    const double v = std::ceil(2.0 * num / (gap * gap) * std::log(2.0 * std::exp(2.0) / delta));
    if (!(v < 4.611686018427388e18)) return fail(XF_EUNSUPPORTED, "trajectory count exceeds 2^62");
    *t = (int64_t)v;
    return ok();
}

}  // extern "C"

namespace {

// Shared by xf_probabilities and xf_probabilities_noalloc.  With noalloc the
// determinant-lemma workspace is the fixed device scratch, no timing events
// are recorded, and nothing is allocated (exact mode then needs the term list
// an earlier call built).
xf_status probabilities_impl(xf_plan *P, const xf_bits128 *d_bits, int64_t B, xf_mode mode, int64_t t,
                             uint64_t seed, double *d_prob, double *d_amp, double *d_logp, void *hip_stream,
                             bool noalloc) {
    if (!plan_valid(P)) return fail(XF_EINVAL, "invalid plan");
    P->fwd_valid = false;   // the workspace may be refilled or reallocated below
    if (B < 0) return fail(XF_EINVAL, "B < 0");
    if (mode != XF_EXACT && mode != XF_RAW_ESTIMATE) return fail(XF_EINVAL, "unknown mode");
    if (mode == XF_RAW_ESTIMATE) {
        if (t < 1) return fail(XF_EINVAL, "t must be >= 1");
        if (t >= (int64_t)1 << 31) return fail(XF_EUNSUPPORTED, "t must be < 2^31");
        if (P->k > 128) return fail(XF_EUNSUPPORTED, "k = %d > 128 in Raw Estimate mode", P->k);
        if (P->keykind < 0) return fail(XF_EUNSUPPORTED, "flip patterns need %d > 63 key bits and k > 63", P->keybits);
    } else if (P->k > 24) {
        return fail(XF_EUNSUPPORTED, "exact mode needs k <= 24 (k = %d)", P->k);
    }
    if (B > 0 && (!d_bits || !d_prob)) return fail(XF_EINVAL, "d_bits or d_prob is NULL");
    if (noalloc && mode == XF_EXACT && P->nxterms < 0 && B > 0)
        return fail(XF_EUNSUPPORTED, "exact mode without allocation needs the term list of an earlier "
                                     "xf_probabilities call with the current parameters");
    DeviceGuard guard(P->device);
    if (!guard.okay) return fail(XF_EDEVICE, "hipSetDevice failed");
    hipStream_t s = (hipStream_t)hip_stream;
    xf::DevPlan d = snapshot(P);
    const bool mixed = P->precision == XF_MIXED;
    const int alg = P->evaluation == XF_EVAL_LU ? 1 : 0;
    // evaluation: the eta <= 16 one-layer lemma kernels, else the general
    // lemma kernel where its sizes fit, else the LU per pattern
    // more than two CPhase layers: the general kernel only (its LU kernel
    // for every bitstring under XF_EVAL_LU)
    const bool multi = P->L >= 3;
    const bool fast = !multi && mode == XF_RAW_ESTIMATE && xf::raw_estimate_uses_lemma(d, alg);
    const bool gen = !fast && (alg == 0 || multi) && xf::gen_applies(d, P->gen);
    const bool all_lu = multi && alg == 1;
    if (multi && !gen)
        return fail(XF_EUNSUPPORTED, "%d CPhase layers: every spin block needs at most 32 input modes and 64 active "
                    "(layer, mode) pairs whose tables fit in LDS", P->L);
    const bool lemma = mode == XF_RAW_ESTIMATE && (fast || gen);   // sampler + evaluation kernels
    // lemma workspace: chunks of bitstrings whose entry regions fit
    uint64_t cap = 0;
    int64_t chunk = B, nchunks = 1;
    uint64_t *ekey = nullptr;
    int2 *ecnt = nullptr;
    uint32_t *ecount = nullptr;
    void *setup = nullptr;   // general lemma: per-bitstring H and base records
    const uint64_t setup_bytes = gen ? (uint64_t)xf::gen_setup_bytes(P->gen) : 0;
    if (lemma && B > 0) {
        cap = xf::lemma_entry_cap(t);
        const uint64_t per_bits = cap * 16 + 4 + setup_bytes;
        if (noalloc) {
            if (per_bits + 256 > xf::kNoAllocScratchBytes)
                return fail(XF_EUNSUPPORTED, "t = %lld needs %llu bytes of scratch per bitstring; the no-allocation "
                            "scratch holds %llu", (long long)t, (unsigned long long)per_bits,
                            (unsigned long long)xf::kNoAllocScratchBytes);
            chunk = std::min<int64_t>(B, (int64_t)((xf::kNoAllocScratchBytes - 256) / per_bits));
        } else {
            chunk = std::min<int64_t>(B, (int64_t)std::max<uint64_t>(1, P->entry_budget / per_bits));
        }
        nchunks = (B + chunk - 1) / chunk;
    }
    // exact mode: flags, then the setup records (and the segments' partial
    // sums), 256-byte aligned
    const uint64_t xflag_bytes = ((uint64_t)B * 4 + 255) & ~(uint64_t)255;
    const uint64_t xpart_bytes =
        (mode == XF_EXACT && gen)
            ? (uint64_t)B * xf::gen_exact_part_segments(B, P->nxterms > 0 ? P->nxterms : ((int64_t)1 << P->k), true) * 64
            : 0;
    if (noalloc && mode == XF_EXACT && gen &&
        xflag_bytes + (uint64_t)B * setup_bytes + xpart_bytes > xf::kNoAllocScratchBytes)
        return fail(XF_EUNSUPPORTED, "B = %lld exceeds the no-allocation scratch in exact mode", (long long)B);
    xf_status st;
    if (!noalloc) {
        if (mode == XF_EXACT && P->nxterms < 0 && B > 0) {
            if (hipStreamSynchronize(s) != hipSuccess) return fail(XF_EDEVICE, "stream synchronisation failed");
            if ((st = build_exact_terms(P, false))) return st;
        }
        if ((st = ensure_events(P, lemma ? 1 + 2 * (size_t)nchunks : 2))) return st;
        if (lemma && B > 0) {
            if ((st = ensure_lemma_workspace(P, chunk, cap, s))) return st;
            ekey = (uint64_t *)P->dekey.p;
            ecnt = (int2 *)P->decnt.p;
            ecount = (uint32_t *)P->decount.p;
        }
        if (mode == XF_EXACT && gen && B > 0 && P->dflags.bytes < (size_t)B * 4) {
            if (hipStreamSynchronize(s) != hipSuccess) return fail(XF_EDEVICE, "stream synchronisation failed");
            if ((st = dev_upload(P->dflags, nullptr, (size_t)B * 4))) return st;
        }
        if (mode == XF_EXACT) ecount = (uint32_t *)P->dflags.p;
        const uint64_t need = (uint64_t)(mode == XF_EXACT ? B : chunk) * setup_bytes + xpart_bytes;
        if (gen && B > 0 && need > 0) {
            if (P->dgsetup.bytes < need) {
                if (hipStreamSynchronize(s) != hipSuccess) return fail(XF_EDEVICE, "stream synchronisation failed");
                if ((st = dev_upload(P->dgsetup, nullptr, need))) return st;
            }
            setup = P->dgsetup.p;
        }
    } else if ((lemma || (mode == XF_EXACT && gen)) && B > 0) {
        void *base = nullptr;
        if (xf::noalloc_scratch(P->device, &base) != hipSuccess)
            return fail(XF_EDEVICE, "could not resolve the device scratch");
        if (lemma) {
            ekey = (uint64_t *)base;
            ecnt = (int2 *)((unsigned char *)base + (size_t)chunk * cap * 8);
            ecount = (uint32_t *)((unsigned char *)base + (size_t)chunk * cap * 16);
            setup = (unsigned char *)base + (((size_t)chunk * (cap * 16 + 4) + 255) & ~(size_t)255);
        } else {
            ecount = (uint32_t *)base;
            setup = (unsigned char *)base + xflag_bytes;
        }
    }
    if (xf::launch_zero_u64((unsigned long long *)P->dnterm.p, s) != hipSuccess)
        return fail(XF_EDEVICE, "launch failed: %s", hipGetErrorString(hipGetLastError()));
    P->last_lemma = 0;
    P->last_gen = 0;
    P->nev = 0;
    if (B == 0) return ok();
    const bool timed = !noalloc;
    hipError_t e = hipSuccess;
    if (timed && hipEventRecord(P->ev[0], s) != hipSuccess) return fail(XF_EDEVICE, "hipEventRecord failed");
    unsigned long long *nterm = (unsigned long long *)P->dnterm.p;
    if (mode == XF_RAW_ESTIMATE) {
        d.scale = std::sqrt(extent_of(P->theta)) / (double)t;
        if (lemma) {
            for (int64_t c = 0; c < nchunks && e == hipSuccess; ++c) {
                const int64_t b0 = c * chunk, nb = std::min(chunk, B - b0);
                hipEvent_t mid = timed ? P->ev[1 + 2 * c] : nullptr;
                if (fast)
                    e = xf::launch_lemma_chunk(d, (const uint64_t *)d_bits, b0, nb, t, seed, ekey, ecnt, ecount, cap,
                                               d_prob, d_amp, d_logp, nterm, mid, s);
                else
                    e = xf::launch_gen_chunk(d, P->gen, mixed, all_lu, (const uint64_t *)d_bits, b0, nb, t, seed, ekey,
                                             ecnt, ecount, cap, setup, d_prob, d_amp, d_logp, nterm, mid, s);
                if (e == hipSuccess && timed) e = hipEventRecord(P->ev[2 + 2 * c], s);
            }
            P->nev = timed ? 1 + 2 * (int)nchunks : 0;
            P->last_lemma = 1;
            P->last_gen = gen ? 1 : 0;
            if (e == hipSuccess && fast && !noalloc && nchunks == 1) {
                P->fwd_valid = true;
                P->fwd_bits = d_bits;
                P->fwd_B = B;
                P->fwd_t = t;
                P->fwd_seed = seed;
            }
        } else {
            e = xf::launch_raw_estimate(d, mixed, (const uint64_t *)d_bits, 0, B, t, seed, d_prob, d_amp, d_logp,
                                        nterm, nullptr, 0, s);
            if (e == hipSuccess && timed) e = hipEventRecord(P->ev[1], s);
            P->nev = timed ? 2 : 0;
        }
    } else {
        if (gen) {
            e = xf::launch_gen_exact(d, P->gen, mixed, all_lu, (const uint64_t *)P->dxkeys.p, (const double2 *)P->dxw.p,
                                     P->nxterms, (const uint64_t *)d_bits, B, ecount, setup, d_prob, d_amp, d_logp,
                                     nterm, nullptr, s,
                                     (P->has_tree && P->evaluation == XF_EVAL_AUTO) ? &P->tree : nullptr);
            P->last_gen = 1;
        } else {
            e = xf::launch_exact(d, mixed, (const uint64_t *)P->dxkeys.p, (const double2 *)P->dxw.p, P->nxterms,
                                 (const uint64_t *)d_bits, B, d_prob, d_amp, d_logp, nterm, nullptr, 0, s);
        }
        if (e == hipSuccess && timed) e = hipEventRecord(P->ev[1], s);
        P->nev = timed ? 2 : 0;
    }
    if (e != hipSuccess) return fail(XF_EDEVICE, "kernel launch failed: %s", hipGetErrorString(e));
    return ok();
}

}  // namespace

extern "C" {

xf_status xf_probabilities(xf_plan *P, const xf_bits128 *d_bits, int64_t B, xf_mode mode, int64_t t,
                           uint64_t seed, double *d_prob, double *d_amp, double *d_logp, void *hip_stream) {
    return probabilities_impl(P, d_bits, B, mode, t, seed, d_prob, d_amp, d_logp, hip_stream, false);
}

xf_status xf_probabilities_noalloc(xf_plan *P, const xf_bits128 *d_bits, int64_t B, xf_mode mode, int64_t t,
                                   uint64_t seed, double *d_prob, double *d_amp, double *d_logp,
                                   void *hip_stream) {
    return probabilities_impl(P, d_bits, B, mode, t, seed, d_prob, d_amp, d_logp, hip_stream, true);
}

}  // extern "C"

namespace {

// The smallest count >= t with at most four significant bits (m 2^e, m < 16).
int64_t round_sig4(int64_t t) {
    if (t < 16) return t;
    const int e = 63 - __builtin_clzll((uint64_t)t) - 3;
    const int64_t m = (t + ((int64_t)1 << e) - 1) >> e;
    return m << e;
}

struct DevScratch {
    void *p = nullptr;
    ~DevScratch() {
        if (p) hipFree(p);
    }
};

}  // namespace

extern "C" {

xf_status xf_estimate(xf_plan *P, const xf_bits128 *d_bits, int64_t B, double eps, double delta, uint64_t seed,
                      double *d_prob, int64_t *h_t, int32_t *h_iterations, void *hip_stream) {
    if (!plan_valid(P)) return fail(XF_EINVAL, "invalid plan");
    if (B < 0) return fail(XF_EINVAL, "B < 0");
    if (!(eps > 0.0 && eps < 1.0) || !(delta > 0.0 && delta < 1.0))
        return fail(XF_EINVAL, "need 0 < eps < 1 and 0 < delta < 1");
    if (B > 0 && (!d_bits || !d_prob)) return fail(XF_EINVAL, "d_bits or d_prob is NULL");
    if (B == 0) {
        if (h_iterations) *h_iterations = 0;
        return ok();
    }
    DeviceGuard guard(P->device);
    if (!guard.okay) return fail(XF_EDEVICE, "hipSetDevice failed");
    hipStream_t s = (hipStream_t)hip_stream;
    std::vector<xf_bits128> hb((size_t)B), gb((size_t)B);
    if (hipMemcpyAsync(hb.data(), d_bits, (size_t)B * sizeof(xf_bits128), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return fail(XF_EDEVICE, "copy of the bitstrings failed");
    DevScratch dbits, dprob;
    if (hipMalloc(&dbits.p, (size_t)B * sizeof(xf_bits128)) != hipSuccess ||
        hipMalloc(&dprob.p, (size_t)B * sizeof(double)) != hipSuccess)
        return fail(XF_ENOMEM, "hipMalloc of %lld bitstrings failed", (long long)B);
    const double xi = extent_of(P->theta);
    std::vector<double> pmax((size_t)B, 1.0), phat((size_t)B, 0.0), gp((size_t)B);
    std::vector<int64_t> tb((size_t)B);
    std::vector<int64_t> order((size_t)B);
    int it = 0;
    for (int i = 1;; ++i) {
        it = i;
        const double eps_i = std::max(eps, std::ldexp(1.0, -i));
        const double delta_i = std::ldexp(delta, -i);
        for (int64_t b = 0; b < B; ++b) {
            int64_t t;
            xf_status st = xf_trajectory_bound(eps_i, delta_i, pmax[b], xi, &t);
            if (st != XF_OK) return st;
            t = round_sig4(t);
            if (t >= (int64_t)1 << 31)
                return fail(XF_EUNSUPPORTED, "Estimate needs t = %lld >= 2^31 trajectories (eps = %g)", (long long)t,
                            eps_i);
            tb[b] = t;
        }
        for (int64_t b = 0; b < B; ++b) order[b] = b;
        std::stable_sort(order.begin(), order.end(), [&](int64_t x, int64_t y) { return tb[x] < tb[y]; });
        for (int64_t j = 0; j < B; ++j) gb[j] = hb[order[j]];
        if (hipMemcpyAsync(dbits.p, gb.data(), (size_t)B * sizeof(xf_bits128), hipMemcpyHostToDevice, s) !=
            hipSuccess)
            return fail(XF_EDEVICE, "upload of the grouped bitstrings failed");
        for (int64_t g0 = 0; g0 < B;) {
            int64_t g1 = g0 + 1;
            while (g1 < B && tb[order[g1]] == tb[order[g0]]) ++g1;
            xf_status st = probabilities_impl(P, (const xf_bits128 *)dbits.p + g0, g1 - g0, XF_RAW_ESTIMATE,
                                              tb[order[g0]], seed + (uint64_t)(i - 1), (double *)dprob.p + g0,
                                              nullptr, nullptr, hip_stream, false);
            if (st != XF_OK) return st;
            g0 = g1;
        }
        if (hipMemcpyAsync(gp.data(), dprob.p, (size_t)B * sizeof(double), hipMemcpyDeviceToHost, s) != hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess)
            return fail(XF_EDEVICE, "download of the estimates failed");
        for (int64_t j = 0; j < B; ++j) phat[order[j]] = gp[j];
        if (eps_i == eps) break;
        for (int64_t b = 0; b < B; ++b) pmax[b] = std::min(pmax[b], std::min(1.0, phat[b] + eps_i));
    }
    if (hipMemcpyAsync(d_prob, phat.data(), (size_t)B * sizeof(double), hipMemcpyHostToDevice, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return fail(XF_EDEVICE, "copy of the results failed");
    if (h_t) std::copy(tb.begin(), tb.end(), h_t);
    if (h_iterations) *h_iterations = it;
    return ok();
}

xf_status xf_circuit_from_gates(int32_t n, int32_t n_gates, const xf_gate *gates, int32_t max_rot, int32_t max_k,
                                double *rot, int32_t *pairs, int32_t *layer, double *theta, int32_t *n_rot,
                                int32_t *k) {
    if (n < 2 || n > 128) return fail(XF_EINVAL, "n must be in [2, 128]");
    if (n_gates < 0 || (n_gates > 0 && !gates)) return fail(XF_EINVAL, "invalid gate list");
    if (!n_rot || !k) return fail(XF_EINVAL, "NULL count output");
    // Pass 1: validate and count layers.  Consecutive matchgates multiply into
    // one rotation layer, consecutive CPhase gates (diagonal, commuting) form
    // one CPhase layer between two rotation layers.
    int nr = 1, nk = 0;
    bool in_cphase = false;
    for (int gi = 0; gi < n_gates; ++gi) {
        const xf_gate &g = gates[gi];
        if (g.kind == XF_GATE_CPHASE) {
            if (g.q0 < 0 || g.q0 >= n || g.q1 < 0 || g.q1 >= n || g.q0 == g.q1)
                return fail(XF_EINVAL, "gate %d: invalid CPhase qubits (%d, %d)", gi, g.q0, g.q1);
            if (!std::isfinite(g.theta) || std::fabs(g.theta) >= 2.0 * M_PI)
                return fail(XF_EINVAL, "gate %d: angle must be finite with |theta| < 2 pi", gi);
            if (!in_cphase) ++nr;
            in_cphase = true;
            ++nk;
        } else if (g.kind == XF_GATE_MATCHGATE) {
            if (g.q0 < 0 || g.q1 != g.q0 + 1 || g.q1 >= n)
                return fail(XF_EINVAL, "gate %d: a matchgate acts on neighbours (q, q + 1) (got %d, %d)", gi, g.q0,
                            g.q1);
            if (!finite_all(&g.g[0][0], 32)) return fail(XF_EINVAL, "gate %d: NaN/Inf entry", gi);
            cd G[4][4];
            for (int r = 0; r < 4; ++r)
                for (int c = 0; c < 4; ++c) G[r][c] = cd(g.g[4 * r + c][0], g.g[4 * r + c][1]);
            // block form of Sec. II-B Eq. 1 with A diagonal (passive: |00>, |11> keep their weight)
            const int zero[10][2] = {{0, 1}, {0, 2}, {0, 3}, {1, 0}, {1, 3}, {2, 0}, {2, 3}, {3, 0}, {3, 1}, {3, 2}};
            for (auto &z : zero)
                if (std::abs(G[z[0]][z[1]]) > 1e-12)
                    return fail(XF_EINVAL, "gate %d: not a particle-number-conserving matchgate (entry %d,%d)", gi,
                                z[0], z[1]);
            for (int r = 0; r < 4; ++r)
                for (int c = 0; c < 4; ++c) {
                    cd v = 0.0;
                    for (int t = 0; t < 4; ++t) v += std::conj(G[t][r]) * G[t][c];
                    if (std::abs(v - (r == c ? 1.0 : 0.0)) > 1e-10) return fail(XF_EINVAL, "gate %d: not unitary", gi);
                }
            const cd detA = G[0][0] * G[3][3], detB = G[1][1] * G[2][2] - G[1][2] * G[2][1];
            if (std::abs(detA - detB) > 1e-10) return fail(XF_EINVAL, "gate %d: det A != det B", gi);
            in_cphase = false;
        } else {
            return fail(XF_EINVAL, "gate %d: unknown kind %d", gi, g.kind);
        }
    }
    *n_rot = nr;   // one more than the runs of CPhase gates (the last layer may be the identity)
    *k = nk;
    if (!rot) return ok();   // sizes only
    if (nr > max_rot || nk > max_k)
        return fail(XF_EINVAL, "the circuit needs %d rotation layers and %d CPhase gates (room for %d and %d)", nr,
                    nk, max_rot, max_k);
    if (nk > 0 && (!pairs || !layer || !theta)) return fail(XF_EINVAL, "NULL CPhase output");
    // Pass 2: fill.  Layer l starts as the identity; a matchgate on (q, q + 1)
    // with vacuum phase a = G[00][00] acts on the modes as the 2 x 2 block
    //   U[q][q] = G[10][10] / a,  U[q][q+1] = G[10][01] / a,
    //   U[q+1][q] = G[01][10] / a,  U[q+1][q+1] = G[01][01] / a
    // (column convention; a_q^dag |0> = |..1_q 0..>, no Jordan-Wigner sign for
    // neighbours; |11> then gets a det U, which is G[11][11] since det A = det B),
    // applied after the layer so far: U_layer <- U_gate U_layer.  The phase a
    // is global and dropped.
    const size_t nn = (size_t)n * n;
    std::vector<cd> U(nn);
    auto reset = [&]() {
        std::fill(U.begin(), U.end(), cd(0.0));
        for (int i = 0; i < n; ++i) U[(size_t)i * n + i] = 1.0;
    };
    int l = 0, j = 0;
    auto flush = [&]() {
        for (size_t i = 0; i < nn; ++i) rot[2 * ((size_t)l * nn + i)] = U[i].real(), rot[2 * ((size_t)l * nn + i) + 1] = U[i].imag();
        ++l;
        reset();
    };
    reset();
    in_cphase = false;
    for (int gi = 0; gi < n_gates; ++gi) {
        const xf_gate &g = gates[gi];
        if (g.kind == XF_GATE_CPHASE) {
            if (!in_cphase) flush();
            in_cphase = true;
            pairs[2 * j] = g.q0;
            pairs[2 * j + 1] = g.q1;
            layer[j] = l - 1;
            theta[j] = g.theta;
            ++j;
        } else {
            in_cphase = false;
            const int q = g.q0;
            auto at = [&](int r, int c) { return cd(g.g[4 * r + c][0], g.g[4 * r + c][1]); };
            const cd a = at(0, 0);
            const cd b00 = at(2, 2) / a, b01 = at(2, 1) / a, b10 = at(1, 2) / a, b11 = at(1, 1) / a;
            for (int c = 0; c < n; ++c) {
                const cd u0 = U[(size_t)q * n + c], u1 = U[(size_t)(q + 1) * n + c];
                U[(size_t)q * n + c] = b00 * u0 + b01 * u1;
                U[(size_t)(q + 1) * n + c] = b10 * u0 + b11 * u1;
            }
        }
    }
    flush();
    return ok();
}

}  // extern "C"

namespace {

// Philox4x32-10 (Salmon et al., SC'11) on the host, for the sampling
// decisions of xf_sample_gates.
void philox_host(const uint32_t ctr_in[4], uint32_t k0, uint32_t k1, uint32_t out[4]) {
    uint32_t c0 = ctr_in[0], c1 = ctr_in[1], c2 = ctr_in[2], c3 = ctr_in[3];
    for (int r = 0; r < 10; ++r) {
        const uint64_t p0 = (uint64_t)0xD2511F53u * c0, p1 = (uint64_t)0xCD9E8D57u * c2;
        const uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0, n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
        c1 = (uint32_t)p1;
        c3 = (uint32_t)p0;
        c0 = n0;
        c2 = n2;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    out[0] = c0, out[1] = c1, out[2] = c2, out[3] = c3;
}

struct PlanHolder {
    xf_plan *p = nullptr;
    ~PlanHolder() {
        if (p) xf_plan_destroy(p);
    }
};

}  // namespace

extern "C" {

xf_status xf_sample_gates(int32_t n, int32_t n_gates, const xf_gate *gates, xf_bits128 input, int64_t S, xf_mode mode,
                          int64_t t, uint64_t seed, xf_precision precision, int device, xf_bits128 *h_samples,
                          void *hip_stream) {
    if (S < 0 || (S > 0 && !h_samples)) return fail(XF_EINVAL, "invalid sample output");
    if (mode != XF_EXACT && mode != XF_RAW_ESTIMATE) return fail(XF_EINVAL, "unknown mode");
    int32_t nr_all = 0, k_all = 0;
    xf_status st = xf_circuit_from_gates(n, n_gates, gates, 0, 0, nullptr, nullptr, nullptr, nullptr, &nr_all,
                                         &k_all);
    if (st != XF_OK) return st;
    for (int64_t s = 0; s < S; ++s) h_samples[s] = input;
    if (S == 0) return ok();
    hipStream_t hs = (hipStream_t)hip_stream;
    DeviceGuard guard(device);
    if (!guard.okay) return fail(XF_EDEVICE, "hipSetDevice(%d) failed", device);
    DevScratch dbits, dprob;
    if (hipMalloc(&dbits.p, (size_t)2 * S * sizeof(xf_bits128)) != hipSuccess ||
        hipMalloc(&dprob.p, (size_t)2 * S * sizeof(double)) != hipSuccess)
        return fail(XF_ENOMEM, "hipMalloc of %lld candidates failed", (long long)(2 * S));
    std::vector<double> rot((size_t)nr_all * n * n * 2), th(std::max(k_all, 1));
    std::vector<int32_t> pairs(2 * std::max(k_all, 1)), layer(std::max(k_all, 1));
    std::vector<xf_bits128> cand((size_t)2 * S);
    std::vector<int64_t> chain((size_t)S);
    std::vector<double> pc((size_t)2 * S);
    PlanHolder plan;
    int32_t plan_nr = -1, plan_k = -1;
    for (int gi = 0; gi < n_gates; ++gi) {
        const xf_gate &g = gates[gi];
        if (g.kind != XF_GATE_MATCHGATE) continue;   // diagonal gates leave the distribution as it is
        // chains whose pair (q, q + 1) holds one particle: two candidates
        const int q = g.q0;
        int64_t na = 0;
        for (int64_t s = 0; s < S; ++s) {
            const xf_bits128 x = h_samples[s];
            const int b0 = (int)((x.w[q >> 6] >> (q & 63)) & 1), b1 = (int)((x.w[(q + 1) >> 6] >> ((q + 1) & 63)) & 1);
            if (b0 + b1 != 1) continue;
            xf_bits128 c10 = x, c01 = x;
            c10.w[q >> 6] |= 1ull << (q & 63);
            c10.w[(q + 1) >> 6] &= ~(1ull << ((q + 1) & 63));
            c01.w[q >> 6] &= ~(1ull << (q & 63));
            c01.w[(q + 1) >> 6] |= 1ull << ((q + 1) & 63);
            cand[2 * na] = c10;
            cand[2 * na + 1] = c01;
            chain[na++] = s;
        }
        if (na == 0) continue;
        // the circuit of gates 0..gi
        int32_t nr = 0, k = 0;
        if ((st = xf_circuit_from_gates(n, gi + 1, gates, nr_all, k_all, rot.data(), pairs.data(), layer.data(),
                                        th.data(), &nr, &k)) != XF_OK)
            return st;
        if (!plan.p || nr != plan_nr || k != plan_k) {
            if (plan.p) xf_plan_destroy(plan.p);
            plan.p = nullptr;
            const xf_circuit c = {n, nr, rot.data(), k, pairs.data(), layer.data(), th.data()};
            if ((st = xf_plan_create(&c, input, precision, device, &plan.p)) != XF_OK) return st;
            plan_nr = nr, plan_k = k;
        } else if ((st = xf_plan_set_params(plan.p, rot.data(), th.data())) != XF_OK) {
            return st;
        }
        if (hipMemcpyAsync(dbits.p, cand.data(), (size_t)2 * na * sizeof(xf_bits128), hipMemcpyHostToDevice, hs) !=
            hipSuccess)
            return fail(XF_EDEVICE, "upload of the candidates failed");
        if ((st = xf_probabilities(plan.p, (const xf_bits128 *)dbits.p, 2 * na, mode, t, seed + (uint64_t)gi,
                                   (double *)dprob.p, nullptr, nullptr, hip_stream)) != XF_OK)
            return st;
        if (hipMemcpyAsync(pc.data(), dprob.p, (size_t)2 * na * sizeof(double), hipMemcpyDeviceToHost, hs) !=
                hipSuccess ||
            hipStreamSynchronize(hs) != hipSuccess)
            return fail(XF_EDEVICE, "download of the candidate probabilities failed");
        for (int64_t a = 0; a < na; ++a) {
            const int64_t s = chain[a];
            const double p10 = pc[2 * a], p01 = pc[2 * a + 1];
            if (!(p10 + p01 > 0.0)) continue;
            const uint32_t ctr[4] = {(uint32_t)s, (uint32_t)gi, 0xFFFFFFFEu, (uint32_t)((uint64_t)s >> 32)};
            uint32_t r[4];
            philox_host(ctr, (uint32_t)seed, (uint32_t)(seed >> 32), r);
            const double u = (double)r[0] * 2.3283064365386963e-10;   // 2^-32
            h_samples[s] = u * (p10 + p01) < p10 ? cand[2 * a] : cand[2 * a + 1];
        }
    }
    return ok();
}

xf_status xf_plan_last_term_count(xf_plan *P, int64_t *count, int64_t *rank_sum) {
    if (!count) return fail(XF_EINVAL, "NULL output");
    xf_work w;
    const xf_status st = xf_plan_last_work(P, &w);
    if (st) return st;
    *count = w.determinants;
    if (rank_sum) *rank_sum = w.rank_sum;
    return ok();
}

xf_status xf_plan_last_work(xf_plan *P, xf_work *work) {
    if (!plan_valid(P) || !work) return fail(XF_EINVAL, "invalid plan or NULL output");
    DeviceGuard guard(P->device);
    if (!guard.okay) return fail(XF_EDEVICE, "hipSetDevice failed");
    unsigned long long v[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    if (hipDeviceSynchronize() != hipSuccess ||
        hipMemcpy(v, P->dnterm.p, 64, hipMemcpyDeviceToHost) != hipSuccess)
        return fail(XF_EDEVICE, "could not read the work counters");
    work->determinants = (int64_t)v[0];
    work->rank_sum = (int64_t)v[1];
    work->flops = (double)v[2];
    work->lemma = P->last_lemma;
    work->backward_lemma = P->last_bwd_lemma;
    work->backward_reused = P->last_bwd_reused;
    work->general = P->last_gen;
    work->fp32_bases = (int64_t)v[3];
    work->philox_blocks = (int64_t)v[4];
    work->tree_bitstrings = (int64_t)v[7];
    work->sample_ms = 0.0;
    work->eval_ms = 0.0;
    for (int i = 1; i < P->nev; ++i) {
        float ms = 0.0f;
        if (hipEventElapsedTime(&ms, P->ev[i - 1], P->ev[i]) != hipSuccess)
            return fail(XF_EDEVICE, "hipEventElapsedTime failed");
        // lemma: odd events close a sampler launch, even ones an evaluation
        if (P->last_lemma && (i & 1)) work->sample_ms += ms;
        else work->eval_ms += ms;
    }
    return ok();
}

xf_status xf_plan_set_workspace_limit(xf_plan *P, uint64_t bytes) {
    if (!plan_valid(P)) return fail(XF_EINVAL, "invalid plan");
    if (bytes == 0) return fail(XF_EINVAL, "workspace limit must be positive");
    P->fwd_valid = false;
    P->entry_budget = bytes;
    return ok();
}

xf_status xf_plan_set_reuse_samples(xf_plan *P, int32_t on) {
    if (!plan_valid(P)) return fail(XF_EINVAL, "invalid plan");
    if (on != 0 && on != 1) return fail(XF_EINVAL, "on must be 0 or 1");
    P->reuse_samples = on == 1;
    P->fwd_valid = false;
    return ok();
}

xf_status xf_plan_set_tree_growth(xf_plan *P, double growth) {
    if (!plan_valid(P)) return fail(XF_EINVAL, "invalid plan");
    if (!(growth > 0.0)) return fail(XF_EINVAL, "growth must be > 0");
    P->tree_growth = growth;
    P->tree.growth2 = growth * growth;
    return ok();
}

xf_status xf_plan_set_mixed_condition(xf_plan *P, double kappa_max) {
    if (!plan_valid(P)) return fail(XF_EINVAL, "invalid plan");
    if (!(kappa_max >= 0.0)) return fail(XF_EINVAL, "kappa_max must be >= 0");
    P->mixed_cond = kappa_max;
    return ok();
}

xf_status xf_plan_set_evaluation(xf_plan *P, xf_evaluation evaluation) {
    if (!plan_valid(P)) return fail(XF_EINVAL, "invalid plan");
    if (evaluation != XF_EVAL_AUTO && evaluation != XF_EVAL_LU && evaluation != XF_EVAL_PATTERNS)
        return fail(XF_EINVAL, "unknown evaluation");
    P->fwd_valid = false;
    P->evaluation = evaluation;
    return ok();
}

xf_status xf_log_prob_backward(xf_plan *P, const xf_bits128 *d_bits, int64_t B, xf_mode mode, int64_t t,
                               uint64_t seed, const double *d_grad_logp, double *h_grad_rot,
                               double *h_grad_theta, void *hip_stream) {
    if (!plan_valid(P)) return fail(XF_EINVAL, "invalid plan");
    if (B < 0) return fail(XF_EINVAL, "B < 0");
    if (mode != XF_EXACT && mode != XF_RAW_ESTIMATE) return fail(XF_EINVAL, "unknown mode");
    if (!h_grad_rot || (P->k > 0 && !h_grad_theta)) return fail(XF_EINVAL, "NULL gradient output");
    if (B > 0 && (!d_bits || !d_grad_logp)) return fail(XF_EINVAL, "d_bits or d_grad_logp is NULL");
    if (P->L > 1) return fail(XF_EUNSUPPORTED, "the backward pass supports at most one CPhase layer");
    if (P->G > 16) return fail(XF_EUNSUPPORTED, "the backward pass supports eta <= 16 (eta = %d)", P->m);
    if (mode == XF_RAW_ESTIMATE) {
        if (t < 1) return fail(XF_EINVAL, "t must be >= 1");
        if (t >= (int64_t)1 << 31) return fail(XF_EUNSUPPORTED, "t must be < 2^31");
        if (P->keykind < 0) return fail(XF_EUNSUPPORTED, "trajectory keys do not fit in 63 bits");
    } else if (P->k > 16) {
        return fail(XF_EUNSUPPORTED, "exact-mode backward needs k <= 16 (k = %d)", P->k);
    }
    const int n = P->n, m = P->m, G = P->G, k = P->k;
    xf::GradLayout lay;
    lay.oP = 0;
    lay.oPhi = n * G;
    lay.oA1 = 2 * n * G;
    lay.oW = lay.oA1 + n * n;
    lay.oG = lay.oW + k;
    lay.stride = lay.oG + 1;
    std::vector<cd> red((size_t)lay.stride, 0.0);
    xf::DevPlan d = snapshot(P);
    const size_t lds = mode == XF_RAW_ESTIMATE ? xf::raw_estimate_bwd_lds_bytes(d, P->precision == XF_MIXED)
                                               : xf::exact_bwd_lds_bytes(d);
    if (lds > 159 * 1024) return fail(XF_EUNSUPPORTED, "backward needs %zu bytes of LDS (k too large)", lds);
    DeviceGuard guard(P->device);
    if (!guard.okay) return fail(XF_EDEVICE, "hipSetDevice failed");
    hipStream_t s = (hipStream_t)hip_stream;
    xf_status st;
    if (B > 0) {
        if (mode == XF_EXACT && (P->nxterms < 0 || !P->xterms_have_dw)) {
            if (hipStreamSynchronize(s) != hipSuccess) return fail(XF_EDEVICE, "stream synchronisation failed");
            if ((st = build_exact_terms(P, true))) return st;
        }
        const bool mixed = P->precision == XF_MIXED;
        const int ngroups = xf::kThreads / G;   // partials per LU-backward workgroup
        const bool lemma = mode == XF_RAW_ESTIMATE && xf::backward_uses_lemma(d, P->evaluation == XF_EVAL_LU ? 1 : 0);
        if (mode == XF_RAW_ESTIMATE) d.scale = std::sqrt(extent_of(P->theta)) / (double)t;
        // partials: [lemma workgroups][LU workgroups x lane groups]
        int64_t chunk = B, nchunks = 1;
        uint64_t cap = 0;
        int n_lemma = 0, n_lu = 0;
        bool reuse = false;   // the forward call's patterns are still in the workspace
        if (lemma) {
            cap = xf::lemma_entry_cap(t);
            const int64_t per = (int64_t)std::max<uint64_t>(1, P->entry_budget / (cap * 16 + 4));
            chunk = std::min<int64_t>(B, per);
            nchunks = (B + chunk - 1) / chunk;
            reuse = P->reuse_samples && P->fwd_valid && nchunks == 1 && P->fwd_bits == (const void *)d_bits &&
                    P->fwd_B == B && P->fwd_t == t && P->fwd_seed == seed;
            // otherwise this call's own samples replace the forward call's
            if (!reuse) P->fwd_valid = false;
            n_lemma = (int)std::min<int64_t>(chunk, 1024);
            n_lu = 64;   // deferred bitstrings only (rare)
            if ((st = ensure_lemma_workspace(P, chunk, cap, s))) return st;
        } else {
            n_lu = (int)std::min<int64_t>(B, 256);
        }
        const int nparts = n_lemma + n_lu * ngroups;
        const size_t part_bytes = (size_t)nparts * lay.stride * 16;
        if ((st = dev_upload(P->dpart, nullptr, part_bytes)) || (st = dev_upload(P->dgsum, nullptr, (size_t)lay.stride * 16)))
            return st;
        hipError_t e = xf::launch_fill_zero((double *)P->dpart.p, part_bytes / 8, s);
        double2 *part = (double2 *)P->dpart.p;
        double2 *part_lu = part + (size_t)n_lemma * lay.stride;
        if (e == hipSuccess) {
            if (lemma) {
                for (int64_t c = 0; c < nchunks && e == hipSuccess; ++c) {
                    const int64_t b0 = c * chunk, nb = std::min(chunk, B - b0);
                    e = xf::launch_lemma_bwd_chunk(d, (const uint64_t *)d_bits, b0, nb, t, seed,
                                                   (uint64_t *)P->dekey.p, (int2 *)P->decnt.p,
                                                   (uint32_t *)P->decount.p, cap, d_grad_logp, part, n_lemma, lay,
                                                   !reuse, s);
                    if (e == hipSuccess)
                        e = xf::launch_raw_estimate_bwd(d, mixed, (const uint64_t *)d_bits, b0, nb, t, seed,
                                                        d_grad_logp, part_lu, n_lu, lay,
                                                        (const uint32_t *)P->decount.p, s);
                }
            } else if (mode == XF_RAW_ESTIMATE) {
                e = xf::launch_raw_estimate_bwd(d, mixed, (const uint64_t *)d_bits, 0, B, t, seed, d_grad_logp,
                                                part_lu, n_lu, lay, nullptr, s);
            } else {
                e = xf::launch_exact_bwd(d, mixed, (const uint64_t *)P->dxkeys.p, (const double2 *)P->dxw.p,
                                         (const double2 *)P->dxdw.p, P->nxterms, (const uint64_t *)d_bits, B,
                                         d_grad_logp, part_lu, n_lu, lay, s);
            }
        }
        if (e == hipSuccess)
            e = xf::launch_reduce_parts(part, nparts, lay.stride, (double2 *)P->dgsum.p, s);
        if (e != hipSuccess) return fail(XF_EDEVICE, "kernel launch failed: %s", hipGetErrorString(e));
        if (hipMemcpyAsync(red.data(), P->dgsum.p, (size_t)lay.stride * 16, hipMemcpyDeviceToHost, s) != hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess)
            return fail(XF_EDEVICE, "could not read back the gradient sums");
        P->last_bwd_lemma = lemma ? 1 : 0;
        P->last_bwd_reused = reuse ? 1 : 0;
    }
    // Host FP64 chain rule from the factors back to rotations and angles.
    // All Gbar below are holomorphic adjoints: dL = 2 Re sum Gbar .* dZ.
    std::vector<cd> GP((size_t)n * m), GPhi((size_t)n * m, 0.0), GA1((size_t)n * n, 0.0);
    for (int r = 0; r < n; ++r)
        for (int a = 0; a < m; ++a) {
            GP[(size_t)r * m + a] = red[lay.oP + (size_t)r * G + a];
            GPhi[(size_t)r * m + a] = red[lay.oPhi + (size_t)r * G + a];
        }
    for (size_t i = 0; i < (size_t)n * n; ++i) GA1[i] = red[lay.oA1 + i];
    std::vector<std::vector<cd>> GR(P->n_rot, std::vector<cd>((size_t)n * n, 0.0));
    std::vector<double> gth(k, 0.0);
    if (P->L == 1) {
        // P = R'_1 Phi0, A1 = R'_1
        std::vector<cd> GRp = GA1;
        const std::vector<cd> &Rp1 = P->Rp[1];
        for (int r = 0; r < n; ++r)
            for (int q = 0; q < n; ++q) {
                cd acc = 0.0;
                for (int a = 0; a < m; ++a) acc += GP[(size_t)r * m + a] * P->hPhi0[(size_t)q * m + a];
                GRp[(size_t)r * n + q] += acc;
            }
        for (int q = 0; q < n; ++q)
            for (int a = 0; a < m; ++a) {
                cd acc = 0.0;
                for (int r = 0; r < n; ++r) acc += Rp1[(size_t)r * n + q] * GP[(size_t)r * m + a];
                GPhi[(size_t)q * m + a] += acc;
            }
        // R'_1 = R_1 D0: Gbar_R1[r][q] = Gbar_R'1[r][q] d_q; angles through d_q
        std::vector<cd> colsum(n, 0.0);
        for (int r = 0; r < n; ++r)
            for (int q = 0; q < n; ++q) {
                GR[1][(size_t)r * n + q] = GRp[(size_t)r * n + q] * P->d0[1][q];
                colsum[q] += GRp[(size_t)r * n + q] * Rp1[(size_t)r * n + q];
            }
        for (int j = 0; j < k; ++j) {
            const cd tr = colsum[P->pairs[2 * j]] + colsum[P->pairs[2 * j + 1]];
            gth[j] += 2.0 * (cd(0.0, 0.5) * tr).real();
        }
    } else {
        // P = Phi0
        for (size_t i = 0; i < GPhi.size(); ++i) GPhi[i] += GP[i];
    }
    for (int r = 0; r < n; ++r)
        for (int a = 0; a < m; ++a) GR[0][(size_t)r * n + P->C[a]] += GPhi[(size_t)r * m + a];
    // weights
    if (mode == XF_EXACT) {
        for (int j = 0; j < k; ++j) gth[j] += 2.0 * red[lay.oW + j].real();
    } else {
        const double gsum = red[lay.oG].real();
        for (int j = 0; j < k; ++j) {
            const double th = P->theta[j];
            const double sg = th > 0.0 ? 1.0 : (th < 0.0 ? -1.0 : 0.0);
            const double sn = std::sin(std::fabs(th) / 4.0), cs = std::cos(std::fabs(th) / 4.0);
            gth[j] += 2.0 * gsum * sg * (cs - sn) / (4.0 * (sn + cs));
        }
    }
    // PyTorch convention: dL/dRe + i dL/dIm = 2 conj(Gbar)
    for (int l = 0; l < P->n_rot; ++l)
        for (size_t i = 0; i < (size_t)n * n; ++i) {
            h_grad_rot[2 * ((size_t)l * n * n + i)] = 2.0 * GR[l][i].real();
            h_grad_rot[2 * ((size_t)l * n * n + i) + 1] = -2.0 * GR[l][i].imag();
        }
    for (int j = 0; j < k; ++j) h_grad_theta[j] = gth[j];
    return ok();
}

xf_status xf_expm_antihermitian(int32_t n, const double *K, double *U) {
    if (n < 1 || n > 128) return fail(XF_EINVAL, "n must be in [1, 128]");
    if (!K || !U) return fail(XF_EINVAL, "NULL pointer");
    if (!finite_all(K, (size_t)n * n * 2)) return fail(XF_EINVAL, "K contains NaN/Inf");
    std::vector<cd> A((size_t)n * n);
    for (size_t i = 0; i < A.size(); ++i) A[i] = cd(K[2 * i], K[2 * i + 1]);
    double scale = 1.0;
    for (const cd &z : A) scale = std::max(scale, std::abs(z));
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j)
            if (std::abs(A[(size_t)i * n + j] + std::conj(A[(size_t)j * n + i])) > 1e-12 * scale)
                return fail(XF_EINVAL, "K is not anti-Hermitian at (%d, %d)", i, j);
    const std::vector<cd> E = expm(A, n);
    for (size_t i = 0; i < E.size(); ++i) U[2 * i] = E[i].real(), U[2 * i + 1] = E[i].imag();
    return ok();
}

xf_status xf_expm_adjoint(int32_t n, const double *K, const double *G_U, double *G_K) {
    if (n < 1 || n > 128) return fail(XF_EINVAL, "n must be in [1, 128]");
    if (!K || !G_U || !G_K) return fail(XF_EINVAL, "NULL pointer");
    if (!finite_all(K, (size_t)n * n * 2) || !finite_all(G_U, (size_t)n * n * 2))
        return fail(XF_EINVAL, "input contains NaN/Inf");
    // L(K^H, G) is the top-right block of exp([[K^H, G], [0, K^H]]).
    const int N2 = 2 * n;
    std::vector<cd> X((size_t)N2 * N2, 0.0);
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) {
            const cd kh = std::conj(cd(K[2 * ((size_t)j * n + i)], K[2 * ((size_t)j * n + i) + 1]));
            X[(size_t)i * N2 + j] = kh;
            X[(size_t)(n + i) * N2 + (n + j)] = kh;
            X[(size_t)i * N2 + (n + j)] = cd(G_U[2 * ((size_t)i * n + j)], G_U[2 * ((size_t)i * n + j) + 1]);
        }
    const std::vector<cd> E = expm(X, N2);
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) {
            const cd v = E[(size_t)i * N2 + (n + j)];
            G_K[2 * ((size_t)i * n + j)] = v.real();
            G_K[2 * ((size_t)i * n + j) + 1] = v.imag();
        }
    return ok();
}

xf_status xf_spin_rotations(int32_t n_layers, int32_t d, const double *K, double *rot) {
    if (n_layers < 1 || d < 1 || d > 64) return fail(XF_EINVAL, "need n_layers >= 1 and 1 <= d <= 64");
    if (!K || !rot) return fail(XF_EINVAL, "NULL pointer");
    const int n = 2 * d;
    std::vector<double> U((size_t)d * d * 2);
    for (int l = 0; l < n_layers; ++l) {
        xf_status st = xf_expm_antihermitian(d, K + (size_t)l * d * d * 2, U.data());
        if (st != XF_OK) return st;
        double *R = rot + (size_t)l * n * n * 2;
        std::fill(R, R + (size_t)n * n * 2, 0.0);
        for (int i = 0; i < d; ++i)
            for (int j = 0; j < d; ++j)
                for (int h = 0; h < 2; ++h) {
                    const size_t o = (size_t)(h * d + i) * n + (h * d + j);
                    R[2 * o] = U[2 * ((size_t)i * d + j)];
                    R[2 * o + 1] = U[2 * ((size_t)i * d + j) + 1];
                }
    }
    return ok();
}

xf_status xf_spin_rotations_adjoint(int32_t n_layers, int32_t d, const double *K, const double *G_rot,
                                    double *G_K) {
    if (n_layers < 1 || d < 1 || d > 64) return fail(XF_EINVAL, "need n_layers >= 1 and 1 <= d <= 64");
    if (!K || !G_rot || !G_K) return fail(XF_EINVAL, "NULL pointer");
    const int n = 2 * d;
    std::vector<double> G((size_t)d * d * 2);
    for (int l = 0; l < n_layers; ++l) {
        // the layer's two diagonal blocks are the same U = exp(K_l): their
        // gradients add
        const double *Gr = G_rot + (size_t)l * n * n * 2;
        for (int i = 0; i < d; ++i)
            for (int j = 0; j < d; ++j)
                for (int c = 0; c < 2; ++c)
                    G[2 * ((size_t)i * d + j) + c] = Gr[2 * ((size_t)i * n + j) + c] +
                                                     Gr[2 * ((size_t)(d + i) * n + (d + j)) + c];
        xf_status st = xf_expm_adjoint(d, K + (size_t)l * d * d * 2, G.data(), G_K + (size_t)l * d * d * 2);
        if (st != XF_OK) return st;
    }
    return ok();
}

xf_status xf_antihermitian_reals_grad(int32_t d, const double *G_K, double *g) {
    if (d < 1 || d > 128) return fail(XF_EINVAL, "d must be in [1, 128]");
    if (!G_K || !g) return fail(XF_EINVAL, "NULL pointer");
    if (!finite_all(G_K, (size_t)d * d * 2)) return fail(XF_EINVAL, "G_K contains NaN/Inf");
    // K_ij = a + i b and K_ji = -a + i b for i < j; K_ii = i c
    const size_t np = (size_t)d * (d - 1) / 2;
    size_t q = 0;
    for (int i = 0; i < d; ++i)
        for (int j = i + 1; j < d; ++j, ++q) {
            const size_t ij = 2 * ((size_t)i * d + j), ji = 2 * ((size_t)j * d + i);
            g[q] = G_K[ij] - G_K[ji];
            g[np + q] = G_K[ij + 1] + G_K[ji + 1];
        }
    for (int i = 0; i < d; ++i) g[2 * np + i] = G_K[2 * ((size_t)i * d + i) + 1];
    return ok();
}

}  // extern "C"
