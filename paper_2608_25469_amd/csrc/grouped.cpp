// Grouped blocked path: many problems with m > 64 advanced together.
//
// Each problem follows exactly the schedule the single-problem blocked path
// gives it (its own I_B from the tuning table, the same diagonal-chunk
// inversions, the same merge products, the same recursive sequence of leaf
// solves and trailing updates), so every result is bit-for-bit the one the
// problem gets alone.  What changes is how the work is launched: the k-th
// operation of every problem goes into one grouped launch, so a batch of
// hundreds of mid-sized solves costs a few dozen launches instead of a few
// dozen per problem.
//
//   1. one zero fill of all diagonal-block workspaces;
//   2. one grouped launch per (data type, diagonal kind, chunk bound) that
//      inverts every diagonal chunk of every problem;
//   3. per merge level, two grouped products (T = C inv(A), then
//      W21 = -inv(D) T) over every pair of every problem at that level;
//   4. per step k of the recursion, grouped products per data type (split by
//      column count so narrow right-hand sides get narrow tiles): the
//      in-order walk of the recursion alternates leaf solve, trailing update,
//      leaf solve, ..., so step k is a leaf for every problem when k is even
//      and an update when k is odd.
// All descriptors of the call go to the device in one copy.

#include <algorithm>
#include <cstring>
#include <vector>

#include "internal.h"

namespace hsma {

size_t blocked_workspace_bytes(bool cx, int64_t m, int ib);
int lookup_block_size(bool cx, int64_t m, int64_t n);
hsma_status upload_async(const void *host, size_t bytes, void *dev, hipStream_t s);
hsma_status launch_inv_group(bool cx, bool unit, int base, const void *items, int count, hipStream_t s);
size_t inv_item_bytes();

namespace {

// Must match InvItem in small_kernels.h (checked at run time by size).
struct InvItem {
    const double *A;
    int64_t lda;
    double *W;
    int32_t ldw, mb;
};

struct Prob {
    bool cx, unit;
    int64_t m, n;
    cplx alpha;
    const double *A;
    int64_t lda;
    double *B;
    int64_t ldb;
    int ib;
    int64_t nb;
    double *W = nullptr, *T = nullptr;  // device addresses (set once allocated)
    size_t ws_off = 0;
    int es() const { return cx ? 2 : 1; }
};

struct Op {
    bool leaf;
    int64_t blk;           // leaf
    int64_t r1, r2, k0;    // update
    bool touched;
};

void walk(const Prob &p, int64_t b0, int64_t nb, bool touched, std::vector<Op> &out) {
    if (nb == 1) {
        out.push_back(Op{true, b0, 0, 0, 0, touched});
        return;
    }
    const int64_t h = nb / 2;
    walk(p, b0, h, touched, out);
    out.push_back(Op{false, 0, (b0 + h) * p.ib, std::min<int64_t>((b0 + nb) * p.ib, p.m), b0 * p.ib,
                     touched});
    walk(p, b0 + h, nb - h, true, out);
}

// A product whose operand addresses are relative to the problem's workspace
// (resolved once the workspace exists) or absolute.
struct Gemm {
    GemmParams g;
    int prob;
    bool a_ws, b_ws, c_ws;  // operand is an offset (in doubles) into the problem's workspace
};

GemmParams make(int M, int N, int K, cplx alpha, const double *A, int64_t lda, const double *B,
                int64_t ldb, cplx beta, double *C, int64_t ldc) {
    GemmParams g{};
    g.M = M;
    g.N = N;
    g.K = K;
    g.A = A;
    g.lda = lda;
    g.B = B;
    g.ldb = ldb;
    g.C = C;
    g.ldc = ldc;
    g.alpha_re = alpha.re;
    g.alpha_im = alpha.im;
    g.beta_re = beta.re;
    g.beta_im = beta.im;
    g.inner = 1;
    return g;
}

const double *off(size_t doubles) { return reinterpret_cast<const double *>(doubles * sizeof(double)); }
double *offw(size_t doubles) { return reinterpret_cast<double *>(doubles * sizeof(double)); }

struct Launch {
    int kind;  // 0 product, 1 chunk inversion
    bool cx = false, unit = false;
    GemmRole role = GemmRole::Update;
    int base = 0;
    size_t img_off = 0;
    int count = 0;
    int64_t tiles = 0;
    int bm = 0, bn = 0;
    double flops = 0;
    std::vector<Gemm> gemms;       // kind 0
    std::vector<InvItem> items;    // kind 1 (W holds workspace offsets until resolved)
    std::vector<int> item_prob;
};

// Merge level `sz` of problem p: the pairs invert_diagonal would form.
void merge_pairs(const Prob &p, int pi, int sz, Launch &l1, Launch &l2) {
    const int es = p.es();
    const int64_t ib = p.ib, lda = p.lda;
    const int64_t nfull = p.m / ib, rem = p.m - nfull * ib;
    int64_t pair = 0;
    auto add = [&](int64_t g, int tsz) {
        const int64_t blk = g / ib, o = g % ib;
        const double *Lc = p.A + es * ((g + sz) + g * lda);
        const size_t wa = es * (blk * ib * ib + o + o * ib);
        const size_t wd = es * (blk * ib * ib + (o + sz) + (o + sz) * ib);
        const size_t w21 = es * (blk * ib * ib + (o + sz) + o * ib);
        const size_t t = (size_t)(p.nb * ib * ib * es) + (size_t)pair * es * sz * sz;
        ++pair;
        Gemm a{make(es * tsz, sz, es * sz, cplx{1.0, 0.0}, Lc, lda, off(wa), es * ib, cplx{0.0, 0.0},
                    offw(t), es * tsz),
               pi, false, true, true};
        Gemm b{make(es * tsz, sz, es * tsz, cplx{-1.0, 0.0}, off(wd), ib, off(t), es * tsz,
                    cplx{0.0, 0.0}, offw(w21), es * ib),
               pi, true, true, true};
        l1.gemms.push_back(a);
        l2.gemms.push_back(b);
    };
    for (int64_t bo = 0; bo < nfull; ++bo)
        for (int64_t bi = 0; bi < ib / (2 * sz); ++bi) add(bo * ib + bi * 2 * sz, sz);
    if (rem > 0) {
        const int64_t g = nfull * ib;
        const int64_t full_pairs = rem / (2 * sz);
        for (int64_t bi = 0; bi < full_pairs; ++bi) add(g + bi * 2 * sz, sz);
        const int64_t a = full_pairs * 2 * sz;
        const int64_t t = rem - a - sz;
        if (t > 0) add(g + a, (int)t);
    }
}

Gemm op_gemm(const Prob &p, int pi, const Op &o) {
    const int es = p.es();
    if (o.leaf) {
        const int64_t r0 = o.blk * p.ib;
        const int mr = (int)std::min<int64_t>(p.ib, p.m - r0);
        double *Br = p.B + es * r0;
        return Gemm{make(es * mr, (int)p.n, es * mr, o.touched ? cplx{1.0, 0.0} : p.alpha,
                         off(es * (size_t)(o.blk * p.ib * p.ib)), p.ib, Br, es * p.ldb,
                         cplx{0.0, 0.0}, Br, es * p.ldb),
                    pi, true, false, false};
    }
    return Gemm{make((int)(es * (o.r2 - o.r1)), (int)p.n, (int)(es * (o.r1 - o.k0)), cplx{-1.0, 0.0},
                     p.A + es * (o.r1 + o.k0 * p.lda), p.lda, p.B + es * o.k0, es * p.ldb,
                     o.touched ? cplx{1.0, 0.0} : p.alpha, p.B + es * o.r1, es * p.ldb),
                pi, false, false, false};
}

}  // namespace

// Enqueue every problem (validated; m > 64; alpha != 0) on stream s.
hsma_status grouped_blocked(const hsma_problem *probs, int64_t count, hipStream_t s) {
    if (count <= 0) return HSMA_SUCCESS;
    if (inv_item_bytes() != sizeof(InvItem)) return HSMA_NOT_SUPPORTED;
    std::vector<Prob> ps;
    ps.reserve(count);
    size_t ws_total = 0;
    for (int64_t i = 0; i < count; ++i) {
        const hsma_problem &q = probs[i];
        Prob p;
        p.cx = q.dtype == HSMA_C64F;
        p.unit = q.diag == HSMA_UNIT;
        p.m = q.m;
        p.n = q.n;
        p.alpha = cplx{q.alpha_re, p.cx ? q.alpha_im : 0.0};
        p.A = static_cast<const double *>(q.A);
        p.lda = q.lda;
        p.B = static_cast<double *>(q.B);
        p.ldb = q.ldb;
        p.ib = lookup_block_size(p.cx, p.m, p.n);
        p.nb = (p.m + p.ib - 1) / p.ib;
        p.ws_off = ws_total;
        ws_total += (blocked_workspace_bytes(p.cx, p.m, p.ib) + 255) / 256 * 256;
        ps.push_back(p);
    }

    std::vector<Launch> launches;
    // 2. chunk inversions, grouped by (dtype, diag, base)
    for (int cxi = 0; cxi < 2; ++cxi)
        for (int ui = 0; ui < 2; ++ui)
            for (int base : {8, 16, 32, 64}) {
                Launch l;
                l.kind = 1;
                l.cx = cxi;
                l.unit = ui;
                l.base = base;
                for (size_t pi = 0; pi < ps.size(); ++pi) {
                    const Prob &p = ps[pi];
                    if (p.cx != (bool)cxi || p.unit != (bool)ui || std::min(p.ib, 64) != base) continue;
                    const int es = p.es();
                    for (int64_t o = 0; o < p.m; o += base) {
                        const int64_t blk = o / p.ib, oo = o % p.ib;
                        InvItem it;
                        it.A = p.A + es * (o + o * p.lda);
                        it.lda = p.lda;
                        it.W = offw(es * (size_t)(blk * p.ib * p.ib + oo + oo * p.ib));
                        it.ldw = p.ib;
                        it.mb = (int32_t)std::min<int64_t>(base, p.m - o);
                        l.items.push_back(it);
                        l.item_prob.push_back((int)pi);
                    }
                }
                if (!l.items.empty()) launches.push_back(std::move(l));
            }
    // 3. merge levels
    for (int sz = 8; sz < 4096; sz *= 2) {
        for (int cxi = 0; cxi < 2; ++cxi) {
            Launch l1, l2;
            l1.kind = l2.kind = 0;
            l1.cx = l2.cx = cxi;
            l1.role = l2.role = GemmRole::Inverse;
            for (size_t pi = 0; pi < ps.size(); ++pi) {
                const Prob &p = ps[pi];
                const int base = std::min(p.ib, 64);
                if (p.cx != (bool)cxi || sz < base || sz >= p.ib) continue;
                // levels run base, 2 base, ... < ib
                int lv = base;
                while (lv < sz) lv *= 2;
                if (lv != sz) continue;
                merge_pairs(p, (int)pi, sz, l1, l2);
            }
            if (!l1.gemms.empty()) {
                launches.push_back(std::move(l1));
                launches.push_back(std::move(l2));
            }
        }
    }
    // 4. recursion steps
    std::vector<std::vector<Op>> ops(ps.size());
    size_t steps = 0;
    for (size_t pi = 0; pi < ps.size(); ++pi) {
        walk(ps[pi], 0, ps[pi].nb, false, ops[pi]);
        steps = std::max(steps, ops[pi].size());
    }
    for (size_t k = 0; k < steps; ++k) {
        for (int cxi = 0; cxi < 2; ++cxi)
            for (int leaf = 1; leaf >= 0; --leaf) {
                Launch l;
                l.kind = 0;
                l.cx = cxi;
                l.role = leaf ? GemmRole::Leaf : GemmRole::Update;
                for (size_t pi = 0; pi < ps.size(); ++pi) {
                    if (ps[pi].cx != (bool)cxi || k >= ops[pi].size() || ops[pi][k].leaf != (bool)leaf)
                        continue;
                    l.gemms.push_back(op_gemm(ps[pi], (int)pi, ops[pi][k]));
                }
                if (!l.gemms.empty()) launches.push_back(std::move(l));
            }
    }

    // Each step's products share one launch whatever their widths: the tile
    // shape follows the widest.  Separate launches for narrow right-hand
    // sides would add kernel boundaries to the dependent chain, and on a
    // served mix (n log-uniform in [1, 512]) cost more than the columns the
    // wide tiles leave idle.

    // Tile shapes, grid sizes and the descriptor image.
    size_t img_bytes = 0;
    for (Launch &l : launches) {
        img_bytes = (img_bytes + 255) / 256 * 256;
        l.img_off = img_bytes;
        if (l.kind == 1) {
            l.count = (int)l.items.size();
            img_bytes += l.items.size() * sizeof(InvItem);
            continue;
        }
        int max_m = 0, max_n = 0;
        for (const Gemm &g : l.gemms) {
            max_m = std::max(max_m, g.g.M);
            max_n = std::max(max_n, g.g.N);
        }
        if (!gemm_grouped_tile(l.role, max_m, max_n, &l.bm, &l.bn)) return HSMA_NOT_SUPPORTED;
        int64_t tiles = 0;
        for (Gemm &g : l.gemms) {
            g.g.tiles_m = (g.g.M + l.bm - 1) / l.bm;
            g.g.tiles_n = (g.g.N + l.bn - 1) / l.bn;
            g.g.tile0 = (int)tiles;
            tiles += (int64_t)g.g.tiles_m * g.g.tiles_n;
            l.flops += 2.0 * g.g.M * (double)g.g.N * g.g.K;
        }
        if (tiles > 0x7fffffff) return HSMA_INVALID_SIZE;
        l.tiles = tiles;
        l.count = (int)l.gemms.size();
        img_bytes += l.gemms.size() * sizeof(GemmParams);
    }
    img_bytes = (img_bytes + 255) / 256 * 256;

    void *dev = nullptr;
    HSMA_TRY(ws_alloc(&dev, img_bytes + ws_total, s));
    unsigned char *base = static_cast<unsigned char *>(dev);
    double *ws = reinterpret_cast<double *>(base + img_bytes);
    for (Prob &p : ps) {
        p.W = reinterpret_cast<double *>(reinterpret_cast<unsigned char *>(ws) + p.ws_off);
    }
    auto resolve = [&](const void *ptr, int pi) {
        return const_cast<double *>(ps[pi].W) + reinterpret_cast<uintptr_t>(ptr) / sizeof(double);
    };
    std::vector<unsigned char> img(img_bytes, 0);
    for (Launch &l : launches) {
        if (l.kind == 1) {
            for (size_t i = 0; i < l.items.size(); ++i) {
                InvItem it = l.items[i];
                it.W = resolve(it.W, l.item_prob[i]);
                std::memcpy(img.data() + l.img_off + i * sizeof(InvItem), &it, sizeof(InvItem));
            }
            continue;
        }
        for (size_t i = 0; i < l.gemms.size(); ++i) {
            GemmParams g = l.gemms[i].g;
            if (l.gemms[i].a_ws) g.A = resolve(g.A, l.gemms[i].prob);
            if (l.gemms[i].b_ws) g.B = resolve(g.B, l.gemms[i].prob);
            if (l.gemms[i].c_ws) g.C = resolve(g.C, l.gemms[i].prob);
            std::memcpy(img.data() + l.img_off + i * sizeof(GemmParams), &g, sizeof(GemmParams));
        }
    }

    hsma_status st = upload_async(img.data(), img.size(), dev, s);
    // 1. zero every diagonal-block workspace (the parts not written by the
    //    chunk inversions must be zero, as in the single-problem path)
    if (st == HSMA_SUCCESS && ws_total > 0)
        st = launch_zero((int64_t)(ws_total / sizeof(double)), 1, 1, ws,
                         (int64_t)(ws_total / sizeof(double)), s);
    for (const Launch &l : launches) {
        if (st != HSMA_SUCCESS) break;
        const void *d = base + l.img_off;
        if (l.kind == 1) {
            ProfScope prof(HSMA_PHASE_DIAG_INV, 0.0, s);
            st = launch_inv_group(l.cx, l.unit, l.base, d, l.count, s);
        } else {
            st = launch_gemm_grouped(l.cx, l.role, l.bm, l.bn, static_cast<const GemmParams *>(d),
                                     l.count, l.tiles, l.flops, s);
        }
    }
    const hsma_status st2 = ws_free(dev, s);
    return st != HSMA_SUCCESS ? st : st2;
}

}  // namespace hsma
