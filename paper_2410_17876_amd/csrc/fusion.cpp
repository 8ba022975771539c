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

template <typename R>
void put_complex(unsigned char* dst, double re, double im) {
    R v[2] = {static_cast<R>(re), static_cast<R>(im)};
    std::memcpy(dst, v, sizeof v);
}

}  // namespace

int build_fused(const int32_t* dims, int n, int precision, const CircuitGate* gates, const std::vector<int>& idx,
                const std::vector<int>& S, int p_low, bool tables, PassPlan* out, std::string* err) {
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
    GatePlan* gp = new GatePlan;
    for (int gi : idx) {
        const CircuitGate& g = gates[gi];
        int32_t lt[QD_MAX_TARGETS], lc[QD_MAX_CONTROLS], lv[QD_MAX_CONTROLS];
        int mi = 0;
        TileGate t;
        std::memset(&t, 0, sizeof t);
        for (int l = 0; l < g.k; ++l) lt[l] = loc[g.targets[l]];
        for (int l = 0; l < g.m; ++l) {
            const int c = g.controls[l];
            if (inS[c]) {
                lc[mi] = loc[c];
                lv[mi] = g.values[l];
                ++mi;
            } else {
                t.oc_stride[t.n_outer] = s[c];
                t.oc_dim[t.n_outer] = (uint32_t)dims[c];
                t.oc_val[t.n_outer] = (uint32_t)g.values[l];
                ++t.n_outer;
            }
        }
        int rc = plan_gate(tdims, nS, lt, g.k, lc, lv, mi, g.U, gp, err);
        if (rc) {
            delete gp;
            return rc;
        }
        if (gp->category == kIdentity) continue;
        if (gp->nseg > kTileMaxSeg) {
            delete gp;
            *err = "tile-local plan has too many segments";
            return QD_ERR_NOT_SUPPORTED;
        }
        t.n_classes = (uint32_t)gp->n_classes;
        t.dec = make_decode<uint32_t, kTileMaxSeg>(*gp);
        t.bases_off = kDecodeBases;
        if (tables) {  // tile-local class bases, decoded once here for every tile
            t.bases_off = (uint32_t)udata.size();
            const Decode<uint64_t> dec = make_decode<uint64_t>(*gp);
            udata.resize(align_up(udata.size() + 2 * (size_t)gp->n_classes, 16));
            uint16_t* b = reinterpret_cast<uint16_t*>(udata.data() + t.bases_off);
            for (uint64_t c = 0; c < gp->n_classes; ++c) b[c] = (uint16_t)decode_base<uint64_t>(dec, c);
        }
        t.u_off = (uint32_t)udata.size();
        if (gp->category == kDense) {
            t.kind = kDense;
            t.M = gp->M;
            for (int a = 0; a < gp->M; ++a) t.off[a] = (uint32_t)gp->off[a];
            udata.resize(udata.size() + (size_t)gp->M * gp->M * ab);
            unsigned char* dst = udata.data() + t.u_off;
            for (int i = 0; i < gp->M * gp->M; ++i) {
                if (precision == kC128) put_complex<double>(dst + i * ab, g.U[2 * i], g.U[2 * i + 1]);
                else put_complex<float>(dst + i * ab, g.U[2 * i], g.U[2 * i + 1]);
            }
        } else {
            t.kind = kMonomial;
            t.M = gp->n_active;
            udata.resize(udata.size() + (size_t)gp->n_active * ab);
            unsigned char* dst = udata.data() + t.u_off;
            for (int i = 0; i < gp->n_active; ++i) {
                t.off[i] = (uint32_t)gp->off[gp->src[i]];
                t.dst[i] = (uint32_t)gp->off[gp->dst[i]];
                if (gp->lam_one[i]) t.one_mask |= 1u << i;
                if (precision == kC128) put_complex<double>(dst + i * ab, gp->lam[2 * i], gp->lam[2 * i + 1]);
                else put_complex<float>(dst + i * ab, gp->lam[2 * i], gp->lam[2 * i + 1]);
            }
        }
        udata.resize(align_up(udata.size(), 16));
        tg.push_back(t);
    }
    delete gp;
    f.ngates = (int)tg.size();
    f.tables = tables;

    // Blob: [TileGate x ngates][gate data][run offsets]. Descriptors' u_off are
    // relative to the start of the gate data; rebase them to the blob start.
    f.gates_off = 0;
    const size_t data_off = align_up(sizeof(TileGate) * tg.size(), 16);
    for (TileGate& t : tg) {
        t.u_off += (uint32_t)data_off;
        if (t.bases_off != kDecodeBases) t.bases_off += (uint32_t)data_off;
    }
    f.run_off_off = align_up(data_off + udata.size(), 16);
    const bool narrow = D < (1ull << 31);
    const size_t ob = narrow ? 4 : 8;
    out->blob.assign(f.run_off_off + R * ob, 0);
    if (!tg.empty()) std::memcpy(out->blob.data(), tg.data(), sizeof(TileGate) * tg.size());
    if (!udata.empty()) std::memcpy(out->blob.data() + data_off, udata.data(), udata.size());
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

    GatePlan* gp = new GatePlan;
    std::vector<int> cur;
    bool inS[QD_MAX_QUDITS] = {false};
    uint64_t prodS = 0;

    auto prod_with = [&](const CircuitGate& g) {
        uint64_t pr = prodS;
        for (int l = 0; l < g.k; ++l)
            if (!inS[g.targets[l]]) pr *= (uint64_t)dims[g.targets[l]];
        return pr;
    };
    auto open_pass = [&]() {
        std::fill(inS, inS + n, false);
        prodS = 1;
        for (int q = 0; q < p_low; ++q) {
            inS[q] = true;
            prodS *= (uint64_t)dims[q];
        }
    };
    auto close_pass = [&]() -> int {
        if (cur.empty()) return QD_OK;
        PassPlan pp;
        if (cur.size() == 1 && !opt.single_as_fused) {
            pp.fused = false;
            pp.gates = cur;
        } else {
            // Pad the tile to the budget with the lowest untouched qudits: fewer,
            // larger workgroups (each has a fixed cost) and longer contiguous runs.
            for (int q = 0; q < n; ++q)
                if (!inS[q] && prodS * (uint64_t)dims[q] <= tile_max) {
                    inS[q] = true;
                    prodS *= (uint64_t)dims[q];
                }
            std::vector<int> S;
            for (int q = 0; q < n; ++q)
                if (inS[q]) S.push_back(q);
            int r2 = build_fused(dims, n, precision, gates, cur, S, p_low, opt.tables, &pp, err);
            if (r2) return r2;
        }
        out.push_back(std::move(pp));
        cur.clear();
        return QD_OK;
    };

    for (int i = 0; i < count; ++i) {
        const CircuitGate& g = gates[i];
        rc = plan_gate(dims, n, g.targets, g.k, g.controls, g.values, g.m, g.U, gp, err);
        if (rc) break;
        if (gp->category == kIdentity) continue;
        const bool can = opt.fuse && fusable(*gp, g.m);
        if (can && !cur.empty() && prod_with(g) <= tile_max) {
            for (int l = 0; l < g.k; ++l)
                if (!inS[g.targets[l]]) {
                    inS[g.targets[l]] = true;
                    prodS *= (uint64_t)dims[g.targets[l]];
                }
            cur.push_back(i);
            continue;
        }
        if ((rc = close_pass())) break;
        if (can) {
            open_pass();
            if (prod_with(g) <= tile_max) {
                for (int l = 0; l < g.k; ++l)
                    if (!inS[g.targets[l]]) {
                        inS[g.targets[l]] = true;
                        prodS *= (uint64_t)dims[g.targets[l]];
                    }
                cur.push_back(i);
                continue;
            }
        }
        PassPlan pp;
        pp.fused = false;
        pp.gates = {i};
        out.push_back(std::move(pp));
    }
    if (!rc) rc = close_pass();
    delete gp;
    if (rc) out.clear();
    return rc;
}

}  // namespace qd
