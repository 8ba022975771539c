// fusion.cpp - split a gate list into HBM passes (fused.h explains a pass).
//
// Greedy and order-preserving: a pass starts with the lowest qudits (enough for
// contiguous runs of at least min_run amplitudes) plus the first gate's targets,
// and takes the following gates while the union of targets keeps the tile within
// tile_max amplitudes. Gates are never reordered, so the fused result is the
// sequential result; inside a tile each gate uses the same per-class arithmetic
// as its one-gate sweep. A gate that cannot join a tile (class larger than 16,
// more than kMaxOuterCtl controls) runs as its own sweep; a pass that ends up
// with one gate is also run as a plain sweep.
#include <algorithm>
#include <cstring>

#include "fusion.h"

namespace qd {

namespace {

bool fusable(const GatePlan& p, int m) {
    if (m > kMaxOuterCtl) return false;
    if (p.category == kDense) return p.M <= kFuseMaxM;
    return p.n_active <= kFuseMaxM;
}

size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

// Same targets in the same order, and the same controls with the same values:
// the two gates act on the same classes with the same local member order.
bool same_classes(const CircuitGate& a, const CircuitGate& b) {
    if (a.k != b.k || a.m != b.m) return false;
    for (int l = 0; l < a.k; ++l)
        if (a.targets[l] != b.targets[l]) return false;
    for (int l = 0; l < a.m; ++l)
        if (a.controls[l] != b.controls[l] || a.values[l] != b.values[l]) return false;
    return true;
}

// Largest dense class a register block takes (its matrix is read into scalar
// registers) and the largest joint class, per precision.
int block_max_m(int precision) { return precision == kC128 ? 4 : 7; }
int block_max_j(int precision) { return precision == kC128 ? kBlockMaxJ128 : kBlockMaxJ; }

// How a gate with this plan (k targets, m controls) enters a register block, or
// -1: uncontrolled dense gates on one or two qudits with small classes, and
// one-qudit phases and cyclic shifts (every factor exactly 1); *shift receives
// the shift.
int block_kind(const GatePlan& p, int k, int m, int precision, int* shift) {
    if (m != 0 || k > 2) return -1;
    if (p.category == kDense) return p.M <= block_max_m(precision) ? (k == 1 ? kBlkDense1 : kBlkDense2) : -1;
    if (k != 1) return -1;
    if (p.category == kDiagonal) return kBlkDiag1;
    if (p.category != kMonomial || p.n_active != p.M) return -1;
    const int sh = ((p.dst[0] - p.src[0]) % p.M + p.M) % p.M;
    for (int j = 0; j < p.n_active; ++j)
        if (!p.lam_one[j] || p.dst[j] != (p.src[j] + sh) % p.M) return -1;
    if (shift) *shift = sh;
    return kBlkShift1;
}

// Whether the device's block switch has a case for this gate code on this block
// shape (fused.hip treats every other code as unreachable).
bool block_code_fits(int shape, int code, int shift, int precision) {
    const int* d = kBlockShapes[shape];
    const int L = d[1] == 1 ? 1 : (d[2] == 1 ? 2 : 3);
    if (d[0] * d[1] * d[2] > block_max_j(precision)) return false;
    const int kind = code / 16, p = (code / 4) % 4, q = code % 4;
    if (code < 0 || p >= L) return false;
    switch (kind) {
        case kBlkDense1: return q == 0 && d[p] <= block_max_m(precision);
        case kBlkDiag1: return q == 0;
        case kBlkShift1: return q == 0 && shift >= 1 && shift < d[p];
        case kBlkDense2: return q < L && q != p && d[p] * d[q] <= block_max_m(precision);
        default: return false;
    }
}

template <typename R>
void put_complex(unsigned char* dst, double re, double im) {
    R v[2] = {static_cast<R>(re), static_cast<R>(im)};
    std::memcpy(dst, v, sizeof v);
}

}  // namespace

int build_fused(const int32_t* dims, int n, int precision, const CircuitGate* gates, const std::vector<int>& idx,
                const std::vector<int>& S, int p_low, PassPlan* out, std::string* err) {
    uint64_t s[QD_MAX_QUDITS];
    s[0] = 1;
    for (int i = 1; i < n; ++i) s[i] = s[i - 1] * (uint64_t)dims[i - 1];
    uint64_t D = s[n - 1] * (uint64_t)dims[n - 1];
    bool inS[QD_MAX_QUDITS] = {false};
    int loc[QD_MAX_QUDITS];
    int32_t tdims[QD_MAX_QUDITS];
    const int nS = (int)S.size();
    uint64_t MS = 1;
    for (int i = 0; i < nS; ++i) {
        inS[S[i]] = true;
        loc[S[i]] = i;
        tdims[i] = dims[S[i]];
        MS *= (uint64_t)dims[S[i]];
    }
    // Runs are as long as the contiguous prefix of S allows.
    int p_run = 0;
    while (p_run < n && inS[p_run]) ++p_run;
    if (p_run < p_low) {
        *err = "fused tile does not hold the low block";
        return QD_ERR_NOT_SUPPORTED;
    }
    p_low = p_run;
    const uint64_t L = p_low < n ? s[p_low] : D;
    const uint64_t R = MS / L;

    FusedLaunch& f = out->launch;
    std::memset(&f, 0, sizeof f);
    f.D = D;
    uint64_t n_tiles = 0;
    if (!free_segments(dims, n, inS, &f.outer_nseg, f.outer_size, f.outer_stride, &n_tiles)) {
        *err = "too many segments outside the tile";
        return QD_ERR_NOT_SUPPORTED;
    }
    f.n_tiles = n_tiles;
    f.tile = (uint32_t)MS;
    f.L = (uint32_t)L;

    const size_t ab = amp_bytes(precision);
    std::vector<TileGate> tg;
    std::vector<unsigned char> udata;
    // Tile-local plans of the pass's gates (identity gates dropped).
    struct Local {
        GatePlan plan;
        TileGate t;
        int k;
        int32_t lt[QD_MAX_TARGETS];
        int in_tile_controls;
        int gi;
    };
    std::vector<Local> locs;
    locs.reserve(idx.size());
    for (int gi : idx) {
        const CircuitGate& g = gates[gi];
        Local L;
        std::memset(&L.t, 0, sizeof L.t);
        int32_t lc[QD_MAX_CONTROLS], lv[QD_MAX_CONTROLS];
        int mi = 0;
        for (int l = 0; l < g.k; ++l) L.lt[l] = loc[g.targets[l]];
        L.k = g.k;
        for (int l = 0; l < g.m; ++l) {
            const int c = g.controls[l];
            if (inS[c]) {
                lc[mi] = loc[c];
                lv[mi] = g.values[l];
                ++mi;
            } else {
                L.t.oc_stride[L.t.n_outer] = s[c];
                L.t.oc_dim[L.t.n_outer] = (uint32_t)dims[c];
                L.t.oc_val[L.t.n_outer] = (uint32_t)g.values[l];
                ++L.t.n_outer;
            }
        }
        L.in_tile_controls = mi;
        L.gi = gi;
        int rc = plan_gate(tdims, nS, L.lt, g.k, lc, lv, mi, g.U, &L.plan, err);
        if (rc) return rc;
        if (L.plan.category == kIdentity) continue;
        locs.push_back(std::move(L));
    }
    auto pairable = [&](const Local& A, const Local& B) {
        if (A.plan.category != kDense || B.plan.category != kDense) return false;
        if (A.in_tile_controls || B.in_tile_controls || A.t.n_outer || B.t.n_outer) return false;
        if (A.plan.M > kPairMaxM || B.plan.M > kPairMaxM || A.k + B.k > QD_MAX_TARGETS) return false;
        for (int i = 0; i < A.k; ++i)
            for (int j = 0; j < B.k; ++j)
                if (A.lt[i] == B.lt[j]) return false;
        return true;
    };
    auto put_u = [&](const double* U, int M) {
        const size_t at = udata.size();
        udata.resize(at + (size_t)M * M * ab);
        unsigned char* dst = udata.data() + at;
        for (int i = 0; i < M * M; ++i) {
            if (precision == kC128) put_complex<double>(dst + i * ab, U[2 * i], U[2 * i + 1]);
            else put_complex<float>(dst + i * ab, U[2 * i], U[2 * i + 1]);
        }
    };
    auto put_classes = [&](TileGate& t, const GatePlan& gp) {  // tile-local class bases, decoded once here
        t.n_classes = (uint32_t)gp.n_classes;
        t.bases_off = (uint32_t)udata.size();
        const Decode<uint64_t> dec = make_decode<uint64_t>(gp);
        udata.resize(align_up(udata.size() + 2 * (size_t)gp.n_classes, 16));
        uint16_t* b = reinterpret_cast<uint16_t*>(udata.data() + t.bases_off);
        for (uint64_t c = 0; c < gp.n_classes; ++c) b[c] = (uint16_t)decode_base<uint64_t>(dec, c);
    };
    // A chain continues while the next gate is dense on the same classes.
    auto chains_with = [&](const Local& A, const Local& B) {
        return A.plan.category == kDense && B.plan.category == kDense && A.plan.M <= kChainMaxM &&
               same_classes(gates[A.gi], gates[B.gi]);
    };
    GatePlan joint;  // geometry of a pair's or a block's joint class
    const int jmax = block_max_j(precision);
    // Block gates: no controls inside the tile (the joint class then holds whole
    // classes of the gate) and at most kBlockMaxOuter outside it (a per-tile test).
    auto in_block = [&](const Local& A) {
        return A.t.n_outer <= kBlockMaxOuter && block_kind(A.plan, A.k, A.in_tile_controls, precision, nullptr) >= 0;
    };
    for (size_t i = 0; i < locs.size(); ++i) {
        Local& A = locs[i];
        TileGate t = A.t;
        // A register block: the longest run of block gates from here whose targets
        // fit one joint class of at most 3 qudits and jmax amplitudes.
        size_t blen = 0;
        std::vector<int> T;  // tile-local qudits of the block
        if (in_block(A)) {
            uint64_t J = 1;
            int nouter = 0;
            while (i + blen < locs.size() && blen < (size_t)kBlockMaxGates && in_block(locs[i + blen])) {
                const Local& B = locs[i + blen];
                if (B.t.n_outer > 0 && nouter == kBlockMaxOuterGates) break;
                std::vector<int> U = T;
                uint64_t JU = J;
                for (int l = 0; l < B.k; ++l)
                    if (std::find(U.begin(), U.end(), B.lt[l]) == U.end()) {
                        U.push_back(B.lt[l]);
                        JU *= (uint64_t)tdims[B.lt[l]];
                    }
                if (U.size() > 3 || JU > (uint64_t)jmax) break;
                T.swap(U);
                J = JU;
                ++blen;
                if (B.t.n_outer > 0) ++nouter;
            }
        }
        if (blen >= 2) {
            // Shape order: dims ascending, ties by tile position.
            std::sort(T.begin(), T.end(), [&](int a, int b) {
                return tdims[a] != tdims[b] ? tdims[a] < tdims[b] : a < b;
            });
            int shape = -1;
            for (int sh = 0; sh < kBlockShapeCount && shape < 0; ++sh) {
                bool same = true;
                for (int p = 0; p < 3; ++p)
                    same = same && kBlockShapes[sh][p] == (p < (int)T.size() ? tdims[T[p]] : 1);
                if (same) shape = sh;
            }
            if (shape < 0) {
                *err = "internal: register block without a shape";
                return QD_ERR_NOT_SUPPORTED;
            }
            int32_t jt[QD_MAX_TARGETS];
            int J = 1;
            for (size_t p = 0; p < T.size(); ++p) {
                jt[p] = T[p];
                J *= tdims[T[p]];
            }
            std::vector<double> eye(2 * (size_t)J * J, 0.0);
            for (int a = 0; a < J; ++a) eye[2 * ((size_t)a * J + a)] = 1.0;
            int rc = plan_gate(tdims, nS, jt, (int)T.size(), nullptr, nullptr, 0, eye.data(), &joint, err);
            if (rc) return rc;
            put_classes(t, joint);
            t.kind = kBlock;
            t.M = J;
            t.M2 = (int32_t)blen;
            t.one_mask = (uint32_t)shape;
            t.n_outer = 0;
            for (int a = 0; a < J; ++a) t.off[a] = (uint32_t)joint.off[a];
            t.u_off = (uint32_t)udata.size();
            t.dst[0] = 0;
            for (size_t j = 0; j < blen; ++j) t.dst[0] += locs[i + j].t.n_outer > 0 ? 1u : 0u;
            const size_t outer_at = t.u_off + blen * sizeof(BlockGate);
            udata.resize(align_up(outer_at + t.dst[0] * sizeof(BlockOuter), 16));
            uint32_t no = 0;
            for (size_t j = 0; j < blen; ++j) {
                const Local& B = locs[i + j];
                const GatePlan& gpl = B.plan;
                if (B.t.n_outer > 0) {
                    BlockOuter bo;
                    std::memset(&bo, 0, sizeof bo);
                    bo.gate = (uint32_t)j;
                    bo.n_outer = B.t.n_outer;
                    for (int l = 0; l < B.t.n_outer; ++l) {
                        bo.oc_stride[l] = B.t.oc_stride[l];
                        bo.oc_dim[l] = B.t.oc_dim[l];
                        bo.oc_val[l] = B.t.oc_val[l];
                        if (D < (1ull << 31)) {
                            bo.oc_sdiv[l] = make_fast_div<uint32_t>(B.t.oc_stride[l]);
                            bo.oc_ddiv[l] = make_fast_div<uint32_t>(B.t.oc_dim[l]);
                        }
                    }
                    std::memcpy(udata.data() + outer_at + (no++) * sizeof(BlockOuter), &bo, sizeof bo);
                }
                BlockGate bg;
                std::memset(&bg, 0, sizeof bg);
                int sh = 0;
                const int kind = block_kind(gpl, B.k, 0, precision, &sh);
                auto pos = [&](int q) { return (int)(std::find(T.begin(), T.end(), q) - T.begin()); };
                bg.code = kind * 16 + pos(B.lt[0]) * 4 + (B.k > 1 ? pos(B.lt[1]) : 0);
                if (!block_code_fits(shape, bg.code, sh, precision)) {
                    *err = "internal: register block gate that its shape does not take";
                    return QD_ERR_NOT_SUPPORTED;
                }
                bg.u_off = (uint32_t)udata.size();
                if (kind == kBlkDense1 || kind == kBlkDense2) {
                    put_u(gates[B.gi].U, gpl.M);
                } else if (kind == kBlkDiag1) {
                    // one factor per local index; identity columns and factors of exactly 1 are kept
                    std::vector<double> lam(2 * (size_t)gpl.M, 0.0);
                    uint32_t om = (1u << gpl.M) - 1;
                    for (int a = 0; a < gpl.M; ++a) lam[2 * a] = 1.0;
                    for (int jj = 0; jj < gpl.n_active; ++jj) {
                        const int a = gpl.src[jj];
                        lam[2 * a] = gpl.lam[2 * jj];
                        lam[2 * a + 1] = gpl.lam[2 * jj + 1];
                        if (!gpl.lam_one[jj]) om &= ~(1u << a);
                    }
                    const size_t at = udata.size();
                    udata.resize(at + (size_t)gpl.M * ab);
                    for (int a = 0; a < gpl.M; ++a) {
                        if (precision == kC128) put_complex<double>(udata.data() + at + a * ab, lam[2 * a], lam[2 * a + 1]);
                        else put_complex<float>(udata.data() + at + a * ab, lam[2 * a], lam[2 * a + 1]);
                    }
                    bg.one_mask = om;
                } else {
                    bg.shift = sh;
                }
                udata.resize(align_up(udata.size(), 16));
                std::memcpy(udata.data() + t.u_off + j * sizeof(BlockGate), &bg, sizeof bg);
            }
            i += blen - 1;
            udata.resize(align_up(udata.size(), 16));
            tg.push_back(t);
            continue;
        }
        size_t len = 1;
        while (i + len < locs.size() && len < (size_t)kChainMaxLen && chains_with(A, locs[i + len])) ++len;
        if (len > 1) {
            const GatePlan& gpl = A.plan;
            put_classes(t, gpl);
            t.kind = kDenseChain;
            t.M = gpl.M;
            t.M2 = (int32_t)len;
            for (int a = 0; a < gpl.M; ++a) t.off[a] = (uint32_t)gpl.off[a];
            t.u_off = (uint32_t)udata.size();
            for (size_t j = 0; j < len; ++j) put_u(gates[locs[i + j].gi].U, gpl.M);
            i += len - 1;
        } else if (i + 1 < locs.size() && pairable(A, locs[i + 1])) {
            // The joint class: targets of the first gate, then of the second (so the
            // joint local index is a1 + M1 a2); U = identity, only the geometry is used.
            const Local& B = locs[i + 1];
            int32_t jt[QD_MAX_TARGETS];
            for (int l = 0; l < A.k; ++l) jt[l] = A.lt[l];
            for (int l = 0; l < B.k; ++l) jt[A.k + l] = B.lt[l];
            const int J = A.plan.M * B.plan.M;
            std::vector<double> eye(2 * (size_t)J * J, 0.0);
            for (int a = 0; a < J; ++a) eye[2 * ((size_t)a * J + a)] = 1.0;
            GatePlan& jp = joint;
            int rc = plan_gate(tdims, nS, jt, A.k + B.k, nullptr, nullptr, 0, eye.data(), &jp, err);
            if (rc) return rc;
            put_classes(t, jp);
            t.kind = kDensePair;
            t.M = A.plan.M;
            t.M2 = B.plan.M;
            for (int a = 0; a < J; ++a) t.off[a] = (uint32_t)jp.off[a];
            t.u_off = (uint32_t)udata.size();
            put_u(gates[A.gi].U, A.plan.M);
            put_u(gates[B.gi].U, B.plan.M);
            ++i;
        } else {
            const GatePlan& gpl = A.plan;
            put_classes(t, gpl);
            t.u_off = (uint32_t)udata.size();
            if (gpl.category == kDense) {
                t.kind = kDense;
                t.M = gpl.M;
                for (int a = 0; a < gpl.M; ++a) t.off[a] = (uint32_t)gpl.off[a];
                put_u(gates[A.gi].U, gpl.M);
            } else {
                t.kind = kMonomial;
                t.M = gpl.n_active;
                udata.resize(udata.size() + (size_t)gpl.n_active * ab);
                unsigned char* dst = udata.data() + t.u_off;
                for (int j = 0; j < gpl.n_active; ++j) {
                    t.off[j] = (uint32_t)gpl.off[gpl.src[j]];
                    t.dst[j] = (uint32_t)gpl.off[gpl.dst[j]];
                    if (gpl.lam_one[j]) t.one_mask |= 1u << j;
                    if (precision == kC128) put_complex<double>(dst + j * ab, gpl.lam[2 * j], gpl.lam[2 * j + 1]);
                    else put_complex<float>(dst + j * ab, gpl.lam[2 * j], gpl.lam[2 * j + 1]);
                }
            }
        }
        udata.resize(align_up(udata.size(), 16));
        tg.push_back(t);
    }
    f.ngates = (int)tg.size();

    // Blob: [TileGate x ngates][gate data][run offsets]. Descriptors' u_off are
    // relative to the start of the gate data; rebase them to the blob start.
    f.gates_off = 0;
    const size_t data_off = align_up(sizeof(TileGate) * tg.size(), 16);
    f.run_off_off = align_up(data_off + udata.size(), 16);
    const bool narrow = D < (1ull << 31);
    const size_t ob = narrow ? 4 : 8;
    out->blob.assign(f.run_off_off + R * ob, 0);
    if (!tg.empty()) std::memcpy(out->blob.data(), tg.data(), sizeof(TileGate) * tg.size());
    if (!udata.empty()) std::memcpy(out->blob.data() + data_off, udata.data(), udata.size());
    // Offsets so far count from the start of the gate data; make them count
    // from the start of the blob.
    rebase_pass_blob(out->blob.data(), f, (uint32_t)data_off, (uint32_t)data_off);
    // Run r enumerates the digits of S above the low block, in increasing qudit order.
    for (uint64_t r = 0; r < R; ++r) {
        uint64_t rest = r, off = 0;
        for (int i = 0; i < nS; ++i) {
            const int q = S[i];
            if (q < p_low) continue;
            off += (rest % (uint64_t)dims[q]) * s[q];
            rest /= (uint64_t)dims[q];
        }
        if (narrow) {
            const uint32_t v = (uint32_t)off;
            std::memcpy(out->blob.data() + f.run_off_off + r * 4, &v, 4);
        } else {
            std::memcpy(out->blob.data() + f.run_off_off + r * 8, &off, 8);
        }
    }
    out->fused = true;
    out->gates = idx;
    return QD_OK;
}

void rebase_pass_blob(unsigned char* blob, const FusedLaunch& f, uint32_t frame, uint32_t delta) {
    TileGate* tg = reinterpret_cast<TileGate*>(blob + f.gates_off);
    for (int g = 0; g < f.ngates; ++g) {
        if (tg[g].kind == kBlock) {
            BlockGate* bg = reinterpret_cast<BlockGate*>(blob + frame + tg[g].u_off);
            for (int j = 0; j < tg[g].M2; ++j) bg[j].u_off += delta;
        }
        tg[g].u_off += delta;
        tg[g].bases_off += delta;
    }
}

int plan_circuit(const int32_t* dims, int n, int precision, const CircuitGate* gates, int count,
                 const CircuitOptions& opt, std::vector<PassPlan>& out, std::string* err) {
    out.clear();
    uint64_t D = 0;
    int rc = check_dims(dims, n, &D, err);
    if (rc) return rc;
    uint64_t s[QD_MAX_QUDITS + 1];
    s[0] = 1;
    for (int i = 0; i < n; ++i) s[i + 1] = s[i] * (uint64_t)dims[i];
    // Low block: the fewest lowest qudits whose block reaches min_run amplitudes.
    int p_low = 0;
    while (p_low < n && s[p_low] < opt.min_run) ++p_low;
    const uint64_t tile_max = opt.tile_max;
    // Upper bound of the pass's device data (descriptor, class-base table of at
    // most tile / 2 classes, matrix): a pass must fit one staging slot.
    const uint64_t tile_bound = std::min<uint64_t>(tile_max, D);

    // Every gate planned once: identity gates are dropped, the others noted with
    // their fusability, device-data bound and qudit masks.
    struct Info {
        bool skip, can, chain;  // chain: dense with a class small enough for a chain
        bool block;             // may join a register block as it is (no controls)
        bool blockU;            // would with its controls dropped (it joins one if they all lie outside the tile)
        size_t bytes;
        uint64_t tmask, cmask;
        uint64_t M;
    };
    std::vector<Info> info(count);
    {
        GatePlan* gp = new GatePlan;
        for (int i = 0; i < count && !rc; ++i) {
            const CircuitGate& g = gates[i];
            rc = plan_gate(dims, n, g.targets, g.k, g.controls, g.values, g.m, g.U, gp, err);
            if (rc) break;
            Info& f = info[i];
            f.skip = gp->category == kIdentity;
            f.can = opt.fuse && fusable(*gp, g.m);
            f.chain = gp->category == kDense && gp->M <= kChainMaxM;
            f.block = block_kind(*gp, g.k, g.m, precision, nullptr) >= 0;
            f.blockU = g.m <= kBlockMaxOuter && block_kind(*gp, g.k, 0, precision, nullptr) >= 0;
            f.M = (uint64_t)gp->M;
            f.bytes = sizeof(TileGate) + (size_t)tile_bound + (size_t)gp->M * gp->M * 16 + 64;
            f.tmask = f.cmask = 0;
            for (int l = 0; l < g.k; ++l) f.tmask |= 1ull << g.targets[l];
            for (int l = 0; l < g.m; ++l) f.cmask |= 1ull << g.controls[l];
        }
        delete gp;
    }
    if (rc) return rc;

    std::vector<char> done(count, 0);
    for (int i = 0; i < count; ++i) done[i] = info[i].skip;
    const uint64_t all = n >= 64 ? ~0ull : (1ull << n) - 1;
    int first = 0;
    while (true) {
        while (first < count && done[first]) ++first;
        if (first >= count) break;
        // Open a pass on the low block and take gates in order while their
        // targets fit the tile. With look-ahead, a gate that does not fit is
        // skipped, and a later gate still joins if it commutes with every
        // skipped gate: its targets meet none of their targets and controls, and
        // its controls meet none of their targets (gates on disjoint qudits, or
        // sharing only control qudits, commute). The scan ends `reorder` gates
        // after the first skipped one, or once every qudit is blocked.
        bool inS[QD_MAX_QUDITS] = {false};
        uint64_t prodS = 1;
        for (int q = 0; q < p_low; ++q) {
            inS[q] = true;
            prodS *= (uint64_t)dims[q];
        }
        std::vector<int> cur;
        size_t blob_est = 0;
        uint64_t blockT = 0, blockA = 0;
        int first_skip = -1;
        for (int j = first; j < count; ++j) {
            if (done[j]) continue;
            if (first_skip >= 0 && j - first_skip > opt.reorder) break;
            const CircuitGate& g = gates[j];
            const Info& f = info[j];
            uint64_t pr = prodS;
            for (int l = 0; l < g.k; ++l)
                if (!inS[g.targets[l]]) pr *= (uint64_t)dims[g.targets[l]];
            const bool fits = f.can && pr <= tile_max && blob_est + f.bytes <= kPassBlobMax;
            const bool commutes = !(f.tmask & blockA) && !(f.cmask & blockT);
            if (fits && commutes) {
                for (int l = 0; l < g.k; ++l) inS[g.targets[l]] = true;
                prodS = pr;
                cur.push_back(j);
                blob_est += f.bytes;
                done[j] = 1;
                continue;
            }
            if (cur.empty()) {  // cannot start a pass (not fusable, or its targets alone exceed the tile)
                PassPlan pp;
                pp.fused = false;
                pp.gates = {j};
                out.push_back(std::move(pp));
                done[j] = 1;
                break;
            }
            if (opt.reorder <= 0) break;
            if (first_skip < 0) first_skip = j;
            blockT |= f.tmask;
            blockA |= f.tmask | f.cmask;
            if ((blockA & all) == all) break;
        }
        if (cur.empty()) continue;
        const bool one_sweep = cur.size() == 1 && !opt.single_as_fused;
        if (!one_sweep) {
            // Pad the tile to the budget with the lowest untouched qudits: fewer,
            // larger workgroups (each has a fixed cost) and longer contiguous runs.
            for (int q = 0; q < n; ++q)
                if (!inS[q] && prodS * (uint64_t)dims[q] <= tile_max) {
                    inS[q] = true;
                    prodS *= (uint64_t)dims[q];
                }
        }
        uint64_t Smask = 0;
        for (int q = 0; q < n; ++q)
            if (inS[q]) Smask |= 1ull << q;
        // A gate may join a register block if it has no controls, or only
        // controls outside the tile (build_fused makes the same test).
        auto blockable = [&](const Info& h) { return h.block || (h.blockU && !(h.cmask & Smask)); };
        if (opt.reorder > 0) {
            // Within the pass, move each chain-sized dense gate back to the last
            // gate on the same classes when it commutes with every gate in
            // between, so that the two share a chain descriptor.
            std::vector<int> seq;
            seq.reserve(cur.size());
            for (int gi : cur) {
                const Info& f = info[gi];
                size_t at = seq.size();
                if (f.chain)
                    for (size_t k = seq.size(); k-- > 0;) {
                        const Info& h = info[seq[k]];
                        if (h.chain && same_classes(gates[seq[k]], gates[gi])) {
                            at = k + 1;
                            break;
                        }
                        if ((f.tmask & (h.tmask | h.cmask)) || (f.cmask & h.tmask)) break;
                    }
                seq.insert(seq.begin() + (std::ptrdiff_t)at, gi);
            }
            cur.swap(seq);
            // Then gather register blocks: a block gate takes every later block gate
            // whose targets still fit its joint class (at most 3 qudits and
            // block_max_j amplitudes) and that commutes with every gate it moves
            // ahead of: its targets meet none of their targets or controls, and its
            // controls (outside the tile, if any) meet none of their targets.
            const uint64_t jmax = (uint64_t)block_max_j(precision);
            std::vector<char> used(cur.size(), 0);
            seq.clear();
            for (size_t a = 0; a < cur.size(); ++a) {
                if (used[a]) continue;
                used[a] = 1;
                seq.push_back(cur[a]);
                const Info& f = info[cur[a]];
                if (!blockable(f)) continue;
                uint64_t T = f.tmask, passA = 0, passT = 0;
                for (size_t b = a + 1; b < cur.size(); ++b) {
                    if (used[b]) continue;
                    const Info& h = info[cur[b]];
                    const uint64_t U = T | h.tmask;
                    uint64_t J = 1;
                    int nq = 0;
                    for (int q = 0; q < n; ++q)
                        if ((U >> q) & 1u) {
                            J *= (uint64_t)dims[q];
                            ++nq;
                        }
                    if (blockable(h) && nq <= 3 && J <= jmax && !(h.tmask & passA) && !(h.cmask & passT)) {
                        used[b] = 1;
                        seq.push_back(cur[b]);
                        T = U;
                    } else {
                        passA |= h.tmask | h.cmask;
                        passT |= h.tmask;
                    }
                }
            }
            cur.swap(seq);
        }
        PassPlan pp;
        if (one_sweep) {
            pp.fused = false;
            pp.gates = cur;
        } else {
            std::vector<int> S;
            for (int q = 0; q < n; ++q)
                if (inS[q]) S.push_back(q);
            rc = build_fused(dims, n, precision, gates, cur, S, p_low, &pp, err);
            if (rc) break;
        }
        out.push_back(std::move(pp));
    }
    if (rc) out.clear();
    return rc;
}

}  // namespace qd
