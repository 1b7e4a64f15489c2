// Host planner: turns the block description of H_sb into the two grouped block-product stages.
//
// H_sb = H_S (x) 1 + 1 (x) H_E + sum_terms coef (A P_S^f) (x) B, and (A (x) B) acts on the
// block coefficient matrix as A X B^T.  For a source block X_b (S sector p, E sector q) and a
// term whose A maps p -> p' and B maps q -> q':
//     Y_{b'} += coef * (-1)^{N(p)} * A[p' <- p] X_b B[q' <- q]^T
// Right products are done first (stage 1):  T_b = X_b [H_E(q)^T | B_1^T | B_2^T | ...]
// then one K-concatenated left product per output block (stage 2):
//     Y_b' = T_b'[:, H_E part] + [H_S(p') | s_1 A_1 | s_2 A_2 | ...] [X_b' ; T part 1 ; ...]
// with the coefficient and the fermion sign of the source folded into the packed A copies.
#include "plan.hpp"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <sstream>

namespace dmrg {

namespace {

std::string load_half(const dmrg_half& h, HalfTable& t, const char* name) {
    std::ostringstream err;
    if (h.nsec <= 0 || !h.qn || !h.dim) {
        err << name << ": no sectors";
        return err.str();
    }
    t.nsec = h.nsec;
    t.nup.resize(h.nsec);
    t.ndn.resize(h.nsec);
    t.dim.resize(h.nsec);
    t.hoff.resize(h.nsec);
    int64_t off = 0;
    for (int p = 0; p < h.nsec; ++p) {
        t.nup[p] = h.qn[2 * p];
        t.ndn[p] = h.qn[2 * p + 1];
        t.dim[p] = h.dim[p];
        if (t.dim[p] <= 0) {
            err << name << ": sector " << p << " has dimension " << t.dim[p];
            return err.str();
        }
        if (p > 0 && !(std::make_pair(t.nup[p - 1], t.ndn[p - 1]) <
                       std::make_pair(t.nup[p], t.ndn[p]))) {
            err << name << ": sectors not strictly increasing at " << p;
            return err.str();
        }
        t.index[{t.nup[p], t.ndn[p]}] = p;
        t.hoff[p] = off;
        off += (int64_t)t.dim[p] * t.dim[p];
    }
    if (!h.H) {
        err << name << ": H missing";
        return err.str();
    }
    t.H.assign(h.H, h.H + off);
    if (h.nop < 0 || (h.nop > 0 && !h.ops)) {
        err << name << ": bad operator list";
        return err.str();
    }
    t.ops.resize(h.nop);
    for (int o = 0; o < h.nop; ++o) {
        auto& op = t.ops[o];
        op.dq[0] = h.ops[o].dq[0];
        op.dq[1] = h.ops[o].dq[1];
        op.boff.assign(h.nsec, -1);
        int64_t boff = 0;
        for (int p = 0; p < h.nsec; ++p) {
            const int p2 = t.find(t.nup[p] + op.dq[0], t.ndn[p] + op.dq[1]);
            if (p2 < 0) continue;
            op.boff[p] = boff;
            boff += (int64_t)t.dim[p2] * t.dim[p];
        }
        if (boff > 0 && !h.ops[o].blocks) {
            err << name << ": operator " << o << " has no blocks";
            return err.str();
        }
        op.data.assign(h.ops[o].blocks, h.ops[o].blocks + boff);
    }
    return "";
}

bool all_zero(const OpRef& r, int rows, int cols) {
    const int64_t cnt = (int64_t)rows * cols;
    for (int64_t i = 0; i < cnt; ++i)
        if (r.data[i] != 0.0) return false;
    return true;
}

OpRef op_from(const HalfTable& t, int opi, bool trans, int src) {
    OpRef r;
    const auto& op = t.ops[opi];
    if (!trans) {
        if (op.boff[src] < 0) return r;
        r.dst = t.find(t.nup[src] + op.dq[0], t.ndn[src] + op.dq[1]);
        r.data = op.data.data() + op.boff[src];
        r.ld = t.dim[r.dst];
        r.transposed = false;
    } else {
        const int pre = t.find(t.nup[src] - op.dq[0], t.ndn[src] - op.dq[1]);
        if (pre < 0 || op.boff[pre] < 0) return r;
        r.dst = pre;
        r.data = op.data.data() + op.boff[pre];
        r.ld = t.dim[src];      // stored block is dim(src) x dim(pre)
        r.transposed = true;
    }
    return r;
}

int round_up(int v, int m) { return (v + m - 1) / m * m; }

// Element offset of (i, k) inside a packed factor with chunk depth ck: i = row (stage 2) or
// column (stage 1), k = K index from the start of the packed K range, nch = chunks per panel,
// per = elements per K index (the bf16 pieces of a split value).  Layout
// [panel][chunk][g][r][piece][t], KPL = ck / 4.
int64_t packed_index(int i, int k, int nch, int ck, int per) {
    const int kpl = ck / 4;
    const int pnl = i / kPanel, r = i % kPanel;
    const int ch = k / ck, g = (k % ck) / kpl, t = k % kpl;
    const int le = kpl * per;
    return (((int64_t)pnl * nch + ch) * 4 + g) * (kPanel * le) + r * le + t;
}

// Reorders a tile list (tiles of one block contiguous) for launch: work groups of `group`
// consecutive tiles, work group i runs on XCD i mod kXcd.  Blocks are assigned to XCDs by
// longest-processing-time on their weights; per XCD the blocks are ordered heaviest first;
// the per-XCD lists are padded with empty tiles (blk = -1) to whole groups and equal length.
template <class T>
std::vector<T> xcd_order(const std::vector<T>& tiles, const std::vector<double>& w, int group) {
    const int nb = (int)w.size();
    std::vector<std::vector<T>> of(nb);
    for (const T& t : tiles) of[t.blk].push_back(t);
    std::vector<int> order(nb);
    for (int i = 0; i < nb; ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return w[a] > w[b]; });
    std::vector<double> load(kXcd, 0.0);
    std::vector<std::vector<T>> lists(kXcd);
    for (int bi : order) {
        if (of[bi].empty()) continue;
        int x = 0;
        for (int i = 1; i < kXcd; ++i)
            if (load[i] < load[x]) x = i;
        load[x] += w[bi];
        lists[x].insert(lists[x].end(), of[bi].begin(), of[bi].end());
    }
    T pad{};
    pad.blk = -1;
    size_t groups = 0;
    for (auto& l : lists) {
        while (l.size() % group) l.push_back(pad);
        groups = std::max(groups, l.size() / group);
    }
    for (auto& l : lists)
        while (l.size() < groups * group) l.push_back(pad);
    std::vector<T> out;
    out.reserve(groups * group * kXcd);
    for (size_t gi = 0; gi < groups; ++gi)
        for (int x = 0; x < kXcd; ++x)
            out.insert(out.end(), lists[x].begin() + gi * group, lists[x].begin() + (gi + 1) * group);
    return out;
}

// Tiles of tm x tn over an M x N block; a last row of tiles with tm / 2 rows or fewer is marked
// half-height (the kernels then run half the row fragments).
void tile_list(std::vector<Tile>& out, int blk, int M, int N, int tm, int tn) {
    for (int m0 = 0; m0 < M; m0 += tm)
        for (int n0 = 0; n0 < N; n0 += tn) out.push_back(Tile{blk, m0, n0, M - m0 <= tm / 2});
}

int cdiv(int a, int b) { return (a + b - 1) / b; }

// K-split family: element offset of row (or column) i, K index k inside a packed operand.
int64_t kpos(const KPack& pk, int i, int k) {
    const int P = i / kKPanel, grp = (i % kKPanel) / 4, x = i % 4;
    const int c = k / 16, b = (k % 16) / 4, kk = k % 4;
    const int lane = 16 * kk + 4 * b + x;
    return pk.off + ((int64_t)P * pk.pstride + (int64_t)c * pk.cstride) * kKPiece +
           (int64_t)(grp / 2) * 128 + lane * 2 + (grp & 1);
}

// Pieces of n groups (of 4 rows or columns): whole runs of 8 groups, then the remainder as
// pieces of 4, 2 and 1 groups (each starting at a multiple of its size).  (start, log2 size).
std::vector<std::pair<int, int>> k_pieces(int ngroups) {
    std::vector<std::pair<int, int>> out;
    int g = 0;
    for (; g + 8 <= ngroups; g += 8) out.push_back({g, 3});
    for (int l = 2; l >= 0; --l)
        if (g + (1 << l) <= ngroups) {
            out.push_back({g, l});
            g += 1 << l;
        }
    return out;
}

}  // namespace

void lds_lists(Plan& P);
void x_lists(Plan& P);
void k_lists(Plan& P);

std::string build_plan(const dmrg_problem* pb, Plan& P) {
    if (!pb) return "problem is NULL";
    std::string e = load_half(pb->S, P.S, "S");
    if (!e.empty()) return e;
    e = load_half(pb->E, P.E, "E");
    if (!e.empty()) return e;
    P.target[0] = pb->target[0];
    P.target[1] = pb->target[1];

    // connection terms: bonds first (four terms each), then generic terms
    if (pb->nbond < 0 || (pb->nbond > 0 && !pb->bonds)) return "bad bond list";
    if (pb->nterm < 0 || (pb->nterm > 0 && !pb->terms)) return "bad term list";
    for (int i = 0; i < pb->nbond; ++i) {
        const dmrg_bond& b = pb->bonds[i];
        for (int s = 0; s < 2; ++s) {
            P.terms.push_back(TermSpec{-b.t, b.opS[s], 0, b.opE[s], 1, 1});   // c+_a c_b
            P.terms.push_back(TermSpec{+b.t, b.opS[s], 1, b.opE[s], 0, 1});   // c+_b c_a
        }
    }
    for (int i = 0; i < pb->nterm; ++i) {
        const dmrg_term& t = pb->terms[i];
        P.terms.push_back(TermSpec{t.coef, t.opS, t.transS ? 1 : 0, t.opE, t.transE ? 1 : 0,
                                   t.fermionic ? 1 : 0});
    }
    for (size_t i = 0; i < P.terms.size(); ++i) {
        const auto& t = P.terms[i];
        if (t.opS < 0 || t.opS >= (int)P.S.ops.size() || t.opE < 0 || t.opE >= (int)P.E.ops.size()) {
            std::ostringstream err;
            err << "term " << i << ": operator index out of range";
            return err.str();
        }
        const int sA = t.transS ? -1 : 1, sB = t.transE ? -1 : 1;
        const auto& a = P.S.ops[t.opS];
        const auto& b = P.E.ops[t.opE];
        if (sA * a.dq[0] + sB * b.dq[0] != 0 || sA * a.dq[1] + sB * b.dq[1] != 0) {
            std::ostringstream err;
            err << "term " << i << ": quantum-number changes of the two factors do not cancel";
            return err.str();
        }
        if (!std::isfinite(t.coef)) return "non-finite term coefficient";
    }

    // psi blocks of the target sector
    P.block_of_S.assign(P.S.nsec, -1);
    int64_t off = 0;
    for (int p = 0; p < P.S.nsec; ++p) {
        const int q = P.E.find(P.target[0] - P.S.nup[p], P.target[1] - P.S.ndn[p]);
        if (q < 0) continue;
        P.block_of_S[p] = (int)P.blocks.size();
        P.blocks.push_back(PsiBlock{p, q, P.S.dim[p], P.E.dim[q], off});
        off += (int64_t)P.S.dim[p] * P.E.dim[q];
    }
    P.n = off;
    if (P.blocks.empty()) return "the target sector is empty";
    const int nb = (int)P.blocks.size();

    // every (term, source block) pair with a non-zero contribution
    P.out_of.assign(nb, {});
    P.into.assign(nb, {});
    for (int bi = 0; bi < nb; ++bi) {
        const auto& B = P.blocks[bi];
        for (size_t ti = 0; ti < P.terms.size(); ++ti) {
            const auto& t = P.terms[ti];
            OpRef a = op_from(P.S, t.opS, t.transS, B.p);
            if (a.dst < 0) continue;
            OpRef b = op_from(P.E, t.opE, t.transE, B.q);
            if (b.dst < 0) continue;
            const int dst = P.block_of_S[a.dst];
            if (dst < 0 || P.blocks[dst].q != b.dst) continue;
            // blocks that are exactly zero contribute nothing and are not counted as work
            if (all_zero(a, P.S.dim[a.dst], B.d) || all_zero(b, P.E.dim[b.dst], B.e)) continue;
            P.edges.push_back(Edge{bi, dst, (int)ti, a, b, 0});
            P.out_of[bi].push_back((int)P.edges.size() - 1);
            P.into[dst].push_back((int)P.edges.size() - 1);
        }
    }

    // stage-1 columns, workspace views (planes padded to whole 32-deep chunks), flops, tiles
    P.N1.assign(nb, 0);
    P.Tview.assign(nb, View{});
    int64_t toff = 0;
    for (int bi = 0; bi < nb; ++bi) {
        const auto& B = P.blocks[bi];
        int N = B.e;
        for (int ei : P.out_of[bi]) {
            P.edges[ei].col = N;
            N += P.blocks[P.edges[ei].dst].e;
        }
        P.N1[bi] = N;
        const int dpad = round_up(B.d, kChunkMax);
        P.Tview[bi] = View{toff, dpad, 2 * dpad, B.d};
        toff += (int64_t)2 * dpad * N;
        P.flops1 += 2.0 * (2 * B.d) * (double)B.e * N;
        tile_list(P.tiles1, bi, 2 * B.d, N, kTile, kTile1N);
        tile_list(P.tiles1n, bi, 2 * B.d, N, kTile, kTile1NN);
    }
    P.T_size = toff;
    std::vector<int> kcat(nb);
    for (int bi = 0; bi < nb; ++bi) {
        const auto& B = P.blocks[bi];
        int k = B.d;
        for (int ei : P.into[bi]) k += P.blocks[P.edges[ei].src].d;
        kcat[bi] = k;
        P.flops2 += 2.0 * B.d * (double)(2 * B.e) * k;
        tile_list(P.tiles2, bi, B.d, 2 * B.e, kTile, kTile);
        tile_list(P.tiles2n, bi, B.d, 2 * B.e, kTile, kTile2NN);
    }
    P.flops_exec = P.flops1 + P.flops2;
    // algorithmic count: the diagonal terms, and per connection term the cheaper of
    // (A X) B^T and A (X B^T) (complex vector: two real planes, two flops per multiply-add)
    P.flops = 0.0;
    for (const auto& B : P.blocks) P.flops += 4.0 * ((double)B.d * B.d * B.e + (double)B.d * B.e * B.e);
    for (const Edge& ed : P.edges) {
        const double d = P.blocks[ed.src].d, e = P.blocks[ed.src].e;
        const double d2 = P.blocks[ed.dst].d, e2 = P.blocks[ed.dst].e;
        P.flops += 4.0 * std::min(d2 * d * e + d2 * e * e2, d * e * e2 + d2 * d * e2);
    }

    // descriptors for both chunk depths
    for (Packing* pk : {&P.pk16, &P.pk32}) {
        pk->ck = (pk == &P.pk16) ? 16 : 32;
        const int ck = pk->ck;
        int64_t roff = 0, aoff = 0;
        for (int bi = 0; bi < nb; ++bi) {
            const auto& B = P.blocks[bi];
            S1Block s;
            s.M = 2 * B.d;
            s.K = B.e;
            s.N = P.N1[bi];
            s.prob = 0;
            s.nch = (B.e + ck - 1) / ck;
            s.pad = 0;
            s.X = View{B.off, P.n, B.d, B.d};
            s.Roff = roff;
            s.T = P.Tview[bi];
            roff += (int64_t)round_up(s.N, kTile1N) * s.nch * ck;
            pk->s1.push_back(s);
        }
        for (int bi = 0; bi < nb; ++bi) {
            const auto& B = P.blocks[bi];
            S2Block s;
            s.M = B.d;
            s.N = 2 * B.e;
            s.prob = 0;
            s.seg0 = (int)pk->segs.size();
            s.Aoff = aoff;
            s.T0 = View{P.Tview[bi].off, P.Tview[bi].poff, P.Tview[bi].ld, B.e};
            s.Y = View{B.off, P.n, B.d, B.e};
            int nch = 0;
            // the diagonal H_S term reads the block itself from the input vector
            pk->segs.push_back(Segment{B.d, 0, 0, 0, View{B.off, P.n, B.d, B.e}});
            nch += (B.d + ck - 1) / ck;
            for (int ei : P.into[bi]) {
                const Edge& ed = P.edges[ei];
                const auto& Bs = P.blocks[ed.src];
                const View& ts = P.Tview[ed.src];
                pk->segs.push_back(Segment{Bs.d, nch, 1, 0,
                                           View{ts.off + (int64_t)ed.col * ts.ld, ts.poff, ts.ld, B.e}});
                nch += (Bs.d + ck - 1) / ck;
            }
            s.nseg = (int)pk->segs.size() - s.seg0;
            s.nch = nch;
            aoff += (int64_t)round_up(B.d, kLTile) * nch * ck;   // whole 64-row tiles
            pk->s2.push_back(s);
        }
        pk->R_elems = roff;
        pk->A_elems = aoff;
    }

    // XCD-aware launch order: every block's tiles go to one XCD (so its packed factor panels
    // and source panels are shared in that XCD's L2), blocks are spread over the XCDs by
    // longest-processing-time, heaviest first inside each XCD.
    std::vector<double> w1(nb), w2(nb);
    for (int bi = 0; bi < nb; ++bi) {
        const auto& B = P.blocks[bi];
        const double nt1 = (double)((2 * B.d + kTile - 1) / kTile) * ((P.N1[bi] + kTile1N - 1) / kTile1N);
        const double nt2 = (double)((B.d + kTile - 1) / kTile) * ((2 * B.e + kTile - 1) / kTile);
        w1[bi] = nt1 * ((B.e + 15) / 16 + 1);
        w2[bi] = nt2 * ((kcat[bi] + 15) / 16 + 2);
    }
    P.tiles1 = xcd_order(P.tiles1, w1, 1);
    P.tiles1n = xcd_order(P.tiles1n, w1, 1);
    P.tiles2 = xcd_order(P.tiles2, w2, 1);
    P.tiles2n = xcd_order(P.tiles2n, w2, 1);
    P.w1 = std::move(w1);
    P.w2 = std::move(w2);
    lds_lists(P);
    x_lists(P);
    k_lists(P);
    P.T_base = P.T_size;
    P.T_size = std::max(P.T_size, P.kf.T_size);
    return "";
}

// Work of the K-split family (internal.hpp): workspace layout, input-vector pieces, block
// descriptors, the stage-2 chunk tables, and tiles of up to 8 x 8 groups of 4 (the edges of each
// plane and column segment covered by pieces of 4, 2 and 1 groups), in XCD order.
void k_lists(Plan& P) {
    KLists& K = P.kf;
    K = KLists{};
    const int nb = (int)P.blocks.size();
    const int ne = (int)P.edges.size();
    auto r32 = [](int v) { return round_up(v, kKPanel); };
    int64_t w = 0;
    std::vector<int64_t> t0(nb);
    for (int bi = 0; bi < nb; ++bi) {
        t0[bi] = w;
        w += (int64_t)P.blocks[bi].d * 2 * r32(P.blocks[bi].e);
    }
    std::vector<KPack> tp(ne);
    for (int ei = 0; ei < ne; ++ei) {
        const int ds = P.blocks[P.edges[ei].src].d, e2 = P.blocks[P.edges[ei].dst].e;
        const int np = 2 * r32(e2) / kKPanel;
        tp[ei] = KPack{w, 1, np};
        w += (int64_t)cdiv(ds, 16) * np * kKPiece;
    }
    for (int bi = 0; bi < nb; ++bi) {
        const auto& B = P.blocks[bi];
        const int dpad = r32(B.d), epad = r32(B.e);
        const int npa = 2 * dpad / kKPanel, nca = cdiv(B.e, 16);
        const int npb = 2 * epad / kKPanel, ncb = cdiv(B.d, 16);
        KXBlock x;
        x.d = B.d;
        x.e = B.e;
        x.prob = 0;
        x.dpad = dpad;
        x.epad = epad;
        x.pad0 = 0;
        x.xoff = B.off;
        x.xplane = P.n;
        x.xa = KPack{w, nca, 1};
        w += (int64_t)npa * nca * kKPiece;
        x.xb = KPack{w, 1, npb};
        w += (int64_t)npb * ncb * kKPiece;
        K.xblk.push_back(x);
        for (int Pn = 0; Pn < npa; ++Pn)
            for (int c = 0; c < nca; ++c) K.pitems.push_back(KPItem{bi, 0, Pn, c});
        for (int Pn = 0; Pn < npb; ++Pn)
            for (int c = 0; c < ncb; ++c) K.pitems.push_back(KPItem{bi, 1, Pn, c});
    }
    K.T_size = w;
    // tiles of a rows x columns range given as (first group, groups) per side
    auto tiles = [](std::vector<KTile>& out, double& wt, int bi, int rg0, int nr, int cg0, int nc,
                    int plane, int seg, int depth) {
        for (auto rp : k_pieces(nr))
            for (auto cp : k_pieces(nc)) {
                out.push_back(KTile{bi, rg0 + rp.first, cg0 + cp.first, 4 * rp.second + cp.second,
                                    plane, seg, 0, 0});
                wt += (double)(1 << rp.second) * (1 << cp.second) * depth;
            }
    };
    std::vector<double> w1(nb, 0.0), w2(nb, 0.0);
    int64_t r = P.pk16.R_elems;
    for (int bi = 0; bi < nb; ++bi) {
        const auto& B = P.blocks[bi];
        const int dpad = r32(B.d), epad = r32(B.e);
        KS1Block s;
        s.edge0 = (int)K.eout.size();
        int N = epad;
        for (int ei : P.out_of[bi]) {
            const int e2 = P.blocks[P.edges[ei].dst].e;
            K.eout.push_back(KEdgeOut{N, e2, r32(e2), 0, tp[ei]});
            N += r32(e2);
        }
        s.M = 2 * dpad;
        s.N = N;
        s.K = B.e;
        s.prob = 0;
        s.d = B.d;
        s.e = B.e;
        s.nch = cdiv(B.e, 16);
        s.nedge = (int)P.out_of[bi].size();
        s.dpad = dpad;
        s.epad = epad;
        s.pad0 = 0;
        s.A = K.xblk[bi].xa;
        s.B = KPack{r, s.nch, 1};
        r += (int64_t)(N / kKPanel) * s.nch * kKPiece;
        s.t0off = t0[bi];
        K.s1.push_back(s);
        for (int pl = 0; pl < 2; ++pl) {
            const int rg0 = pl * dpad / 4, nr = cdiv(B.d, 4);
            tiles(K.t1, w1[bi], bi, rg0, nr, 0, cdiv(B.e, 4), pl, -1, s.nch + 2);
            for (int k = 0; k < s.nedge; ++k) {
                const KEdgeOut& eo = K.eout[s.edge0 + k];
                tiles(K.t1, w1[bi], bi, rg0, nr, eo.col / 4, cdiv(eo.e2, 4), pl, k, s.nch + 2);
            }
        }
    }
    K.R_elems = r - P.pk16.R_elems;
    int64_t a = P.pk16.A_elems;
    for (int bi = 0; bi < nb; ++bi) {
        const auto& B = P.blocks[bi];
        const int epad = r32(B.e);
        KS2Block s;
        s.M = B.d;
        s.N = 2 * epad;
        s.prob = 0;
        s.ctab0 = (int)K.ctab.size();
        s.e = B.e;
        s.epad = epad;
        s.pad0 = 0;
        const int npb = 2 * epad / kKPanel;
        for (int c = 0; c < cdiv(B.d, 16); ++c)
            K.ctab.push_back(K.xblk[bi].xb.off + (int64_t)c * npb * kKPiece);
        for (int ei : P.into[bi]) {
            const int ds = P.blocks[P.edges[ei].src].d;
            for (int c = 0; c < cdiv(ds, 16); ++c)
                K.ctab.push_back(tp[ei].off + (int64_t)c * tp[ei].cstride * kKPiece);
        }
        s.nch = (int)K.ctab.size() - s.ctab0;
        s.A = KPack{a, s.nch, 1};
        a += (int64_t)cdiv(B.d, kKPanel) * s.nch * kKPiece;
        s.t0off = t0[bi];
        s.Y = View{B.off, P.n, B.d, B.e};
        K.s2.push_back(s);
        for (int pl = 0; pl < 2; ++pl)
            tiles(K.t2, w2[bi], bi, 0, cdiv(B.d, 4), pl * epad / 4, cdiv(B.e, 4), pl, -1,
                  s.nch / 4 + 3);
    }
    K.A_elems = a - P.pk16.A_elems;
    K.t1 = xcd_order(K.t1, w1, 1);
    K.t2 = xcd_order(K.t2, w2, 1);
}

// Work of the LDS-staged family: the chunk table of every stage-2 block (its segments' source
// views, 16-deep chunks), 64 x 32 output tiles, those with more than kXSplitChunks chunks cut
// into two slices of about equal length, and the output regions of the cut tiles.
void x_lists(Plan& P) {
    Packing& pk = P.pk16;
    pk.xch.clear();
    pk.x2.clear();
    pk.xz.clear();
    const int nb = (int)P.blocks.size();
    std::vector<double> w(nb, 0.0);
    std::vector<int> ctab0(nb, 0);
    for (int bi = 0; bi < nb; ++bi) {
        const S2Block& s = pk.s2[bi];
        ctab0[bi] = (int)pk.xch.size();
        for (int si = 0; si < s.nseg; ++si) {
            const Segment& sg = pk.segs[s.seg0 + si];
            const int nc = (sg.K + pk.ck - 1) / pk.ck;
            for (int c = 0; c < nc; ++c)
                pk.xch.push_back(XChunk{sg.B.off - (int64_t)sg.ch0 * pk.ck, sg.B.poff, sg.B.ld, sg.src});
        }
    }
    auto panels = [](int v) { return (v + kPanel - 1) / kPanel; };
    for (int bi = 0; bi < nb; ++bi) {
        const S2Block& s = pk.s2[bi];
        const bool split = s.nch > kXSplitChunks;
        const int half = s.nch / 2;
        for (int m0 = 0; m0 < s.M; m0 += kLTile)
            for (int n0 = 0; n0 < s.N; n0 += kXTile2N) {
                const double area = (double)std::min(4, panels(s.M - m0)) *
                                    std::min(2, panels(s.N - n0));
                if (split) {
                    pk.x2.push_back(XItem2{bi, m0, n0, 0, half, 1, ctab0[bi], 0});
                    pk.x2.push_back(XItem2{bi, m0, n0, half, s.nch, 2, ctab0[bi], 0});
                    pk.xz.push_back(XZero{bi, m0, n0, 0});
                } else {
                    pk.x2.push_back(XItem2{bi, m0, n0, 0, s.nch, 0, ctab0[bi], 0});
                }
                w[bi] += area * (s.nch + 2);
            }
    }
    pk.x2 = xcd_order(pk.x2, w, 1);
    for (const XItem2& t : pk.x2)
        if (t.kc1 - t.kc0 > kXMaxItemChunks) {   // the family needs every item's table in LDS
            pk.x2.clear();
            pk.xz.clear();
            break;
        }
}

// Work lists of the LDS-tiled kernels: 64 x 64 tiles; stage-2 tiles whose K exceeds a slice
// are cut into about equal slices of at most `slice` chunks (partial tiles plus a reduction).
void lds_lists(Plan& P) {
    const int nb = (int)P.blocks.size();
    auto panels = [](int v) { return (v + kPanel - 1) / kPanel; };
    std::vector<double> w(nb, 0.0);
    P.l1.clear();
    for (int bi = 0; bi < nb; ++bi) {
        const S1Block& s = P.pk16.s1[bi];
        for (int m0 = 0; m0 < s.M; m0 += kLTile)
            for (int n0 = 0; n0 < s.N; n0 += kLTile) {
                P.l1.push_back(LItem1{bi, m0, n0, 0});
                w[bi] += (double)std::min(4, panels(s.M - m0)) * std::min(4, panels(s.N - n0)) *
                         (s.nch + 1);
            }
    }
    P.l1 = xcd_order(P.l1, w, 1);
    for (Packing* pk : {&P.pk16, &P.pk32}) {
        pk->slice = pk->ck == 16 ? kLSlice : kLSlice / 2;   // chunks: K = 256 either way
        pk->l2.clear();
        pk->lred.clear();
        pk->nslots = 0;
        std::fill(w.begin(), w.end(), 0.0);
        for (int bi = 0; bi < nb; ++bi) {
            const S2Block& s = pk->s2[bi];
            const int nsl = std::max(1, (s.nch + pk->slice - 1) / pk->slice);
            for (int m0 = 0; m0 < s.M; m0 += kLTile)
                for (int n0 = 0; n0 < s.N; n0 += kLTile) {
                    const double area = (double)std::min(4, panels(s.M - m0)) *
                                        std::min(4, panels(s.N - n0));
                    if (nsl == 1) {
                        pk->l2.push_back(LItem2{bi, m0, n0, 0, s.nch, -1});
                    } else {
                        pk->lred.push_back(LRed{bi, m0, n0, pk->nslots, nsl, 0});
                        for (int q = 0; q < nsl; ++q)
                            pk->l2.push_back(LItem2{bi, m0, n0, (int)((int64_t)s.nch * q / nsl),
                                                    (int)((int64_t)s.nch * (q + 1) / nsl),
                                                    pk->nslots++});
                    }
                    w[bi] += area * (s.nch + nsl);
                }
        }
        pk->l2 = xcd_order(pk->l2, w, 1);
    }
}

void merge_plans(const std::vector<const Plan*>& plans, Merged& out) {
    out = Merged{};
    std::vector<Tile> t1, t1n, t2, t2n;
    std::vector<double> w1, w2;
    std::vector<LItem1> l1;
    std::vector<LItem2> l2[2];
    std::vector<XItem2> x2;
    int boff = 0;
    for (size_t i = 0; i < plans.size(); ++i) {
        const Plan& P = *plans[i];
        const Packing* pks[2] = {&P.pk16, &P.pk32};
        for (int k = 0; k < 2; ++k) {
            const int soff = (int)out.segs[k].size();
            for (S1Block b : pks[k]->s1) {
                b.prob = (int)i;
                out.s1[k].push_back(b);
            }
            for (S2Block b : pks[k]->s2) {
                b.prob = (int)i;
                b.seg0 += soff;
                out.s2[k].push_back(b);
            }
            out.segs[k].insert(out.segs[k].end(), pks[k]->segs.begin(), pks[k]->segs.end());
        }
        for (Tile t : P.tiles1)
            if (t.blk >= 0) t1.push_back(Tile{t.blk + boff, t.m0, t.n0, t.half});
        for (Tile t : P.tiles1n)
            if (t.blk >= 0) t1n.push_back(Tile{t.blk + boff, t.m0, t.n0, t.half});
        for (Tile t : P.tiles2)
            if (t.blk >= 0) t2.push_back(Tile{t.blk + boff, t.m0, t.n0, t.half});
        for (Tile t : P.tiles2n)
            if (t.blk >= 0) t2n.push_back(Tile{t.blk + boff, t.m0, t.n0, t.half});
        w1.insert(w1.end(), P.w1.begin(), P.w1.end());
        w2.insert(w2.end(), P.w2.begin(), P.w2.end());
        for (LItem1 t : P.l1)
            if (t.blk >= 0) {
                t.blk += boff;
                l1.push_back(t);
            }
        {
            const int coff = (int)out.xch.size();
            out.xch.insert(out.xch.end(), P.pk16.xch.begin(), P.pk16.xch.end());
            for (XItem2 t : P.pk16.x2)
                if (t.blk >= 0) {
                    t.blk += boff;
                    t.ctab0 += coff;
                    x2.push_back(t);
                }
            for (XZero z : P.pk16.xz) {
                z.blk += boff;
                out.xz.push_back(z);
            }
        }
        for (int k = 0; k < 2; ++k) {
            const int soff = out.nslots[k];
            for (LItem2 t : pks[k]->l2)
                if (t.blk >= 0) {
                    t.blk += boff;
                    if (t.slot >= 0) t.slot += soff;
                    l2[k].push_back(t);
                }
            for (LRed r : pks[k]->lred) {
                r.blk += boff;
                r.slot0 += soff;
                out.lred[k].push_back(r);
            }
            out.nslots[k] += pks[k]->nslots;
        }
        boff += (int)P.blocks.size();
    }
    out.tiles1 = xcd_order(t1, w1, 1);
    out.tiles1n = xcd_order(t1n, w1, 1);
    out.tiles2 = xcd_order(t2, w2, 1);
    out.tiles2n = xcd_order(t2n, w2, 1);
    // the LDS lists keep each problem's block order: weights by tiles of the merged lists
    std::vector<double> wl(boff, 0.0);
    for (const LItem1& t : l1) wl[t.blk] += 1.0;
    out.l1 = xcd_order(l1, wl, 1);
    for (int k = 0; k < 2; ++k) {
        std::fill(wl.begin(), wl.end(), 0.0);
        for (const LItem2& t : l2[k]) wl[t.blk] += (double)(t.kc1 - t.kc0 + 1);
        out.l2[k] = xcd_order(l2[k], wl, 1);
    }
    std::fill(wl.begin(), wl.end(), 0.0);
    for (const XItem2& t : x2) wl[t.blk] += (double)(t.kc1 - t.kc0 + 2);
    out.x2 = xcd_order(x2, wl, 1);
}

namespace {

uint16_t bf16_rne(float f) {
    uint32_t u;
    std::memcpy(&u, &f, 4);
    if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40);   // NaN
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

float bf16_to_float(uint16_t h) {
    const uint32_t u = (uint32_t)h << 16;
    float f;
    std::memcpy(&f, &u, 4);
    return f;
}

// Writes value v at packed position (i, k) in the arithmetic `kind` (offsets of the
// descriptors count one element per K index; a split value occupies `per` elements).
struct Writer {
    int kind, ck, per;
    uint8_t* base;
    void put(int64_t blk_off, int i, int k, int nch, double v) const {
        const int64_t o = blk_off * per + packed_index(i, k, nch, ck, per);
        if (kind == DMRG_FP64) {
            reinterpret_cast<double*>(base)[o] = v;
        } else if (kind == DMRG_FP32) {
            reinterpret_cast<float*>(base)[o] = (float)v;
        } else {
            // x = piece_0 + piece_1 (+ piece_2) + residual, each piece the bf16 rounding of
            // what the previous ones leave
            float rest = (float)v;
            uint16_t* b = reinterpret_cast<uint16_t*>(base);
            for (int q = 0; q < per; ++q) {
                const uint16_t h = bf16_rne(rest);
                b[o + q * (ck / 4)] = h;
                rest -= bf16_to_float(h);
            }
        }
    }
};

}  // namespace

void pack_operators(const Plan& P, int kind, std::vector<uint8_t>& A, std::vector<uint8_t>& R) {
    const bool split = kind == DMRG_BF16X3 || kind == DMRG_BF16X6;
    const Packing& pk = split ? P.pk32 : P.pk16;
    const size_t esz = (kind == DMRG_FP64) ? 8 : (kind == DMRG_FP32 ? 4 : 2);
    const int per = kind == DMRG_BF16X3 ? 2 : (kind == DMRG_BF16X6 ? 3 : 1);
    const bool kfam = kind == DMRG_FP64;   // the K-split family's packs follow (FP64 only)
    A.assign((size_t)(pk.A_elems + (kfam ? P.kf.A_elems : 0)) * per * esz, 0);
    R.assign((size_t)(pk.R_elems + (kfam ? P.kf.R_elems : 0)) * per * esz, 0);
    const Writer wa{kind, pk.ck, per, A.data()}, wr{kind, pk.ck, per, R.data()};
    const int nb = (int)P.blocks.size();
    for (int bi = 0; bi < nb; ++bi) {
        const auto& B = P.blocks[bi];
        // R_b (K = e rows, N columns): R(k, j) = H_E(q)(j, k), then R(k, col + j) = B(j, k)
        const S1Block& s1 = pk.s1[bi];
        const double* HE = P.E.H.data() + P.E.hoff[B.q];
        for (int j = 0; j < B.e; ++j)
            for (int k = 0; k < B.e; ++k) wr.put(s1.Roff, j, k, s1.nch, HE[(int64_t)k * B.e + j]);
        for (int ei : P.out_of[bi]) {
            const Edge& ed = P.edges[ei];
            const int e2 = P.blocks[ed.dst].e;
            for (int j = 0; j < e2; ++j)
                for (int k = 0; k < B.e; ++k) wr.put(s1.Roff, ed.col + j, k, s1.nch, ed.b.at(j, k));
        }
        // Acat_b (d rows): [H_S(p) | coef * sign * A per incoming term], segments chunk-aligned
        const S2Block& s2 = pk.s2[bi];
        const double* HS = P.S.H.data() + P.S.hoff[B.p];
        for (int k = 0; k < B.d; ++k)
            for (int i = 0; i < B.d; ++i) wa.put(s2.Aoff, i, k, s2.nch, HS[(int64_t)k * B.d + i]);
        int si = 1;
        for (int ei : P.into[bi]) {
            const Edge& ed = P.edges[ei];
            const auto& Bs = P.blocks[ed.src];
            const auto& t = P.terms[ed.term];
            const double c = t.coef * (t.fermionic ? P.S.parity(Bs.p) : 1);
            const int kbase = pk.segs[s2.seg0 + si].ch0 * pk.ck;
            for (int k = 0; k < Bs.d; ++k)
                for (int i = 0; i < B.d; ++i) wa.put(s2.Aoff, i, kbase + k, s2.nch, c * ed.a.at(i, k));
            ++si;
        }
    }
    if (!kfam) return;
    double* KA = reinterpret_cast<double*>(A.data());
    double* KR = reinterpret_cast<double*>(R.data());
    for (int bi = 0; bi < nb; ++bi) {
        const auto& B = P.blocks[bi];
        const KS1Block& s1 = P.kf.s1[bi];
        const double* HE = P.E.H.data() + P.E.hoff[B.q];
        for (int j = 0; j < B.e; ++j)
            for (int k = 0; k < B.e; ++k) KR[kpos(s1.B, j, k)] = HE[(int64_t)k * B.e + j];
        for (int k2 = 0; k2 < s1.nedge; ++k2) {
            const Edge& ed = P.edges[P.out_of[bi][k2]];
            const KEdgeOut& eo = P.kf.eout[s1.edge0 + k2];
            for (int j = 0; j < eo.e2; ++j)
                for (int k = 0; k < B.e; ++k) KR[kpos(s1.B, eo.col + j, k)] = ed.b.at(j, k);
        }
        const KS2Block& s2 = P.kf.s2[bi];
        const double* HS = P.S.H.data() + P.S.hoff[B.p];
        for (int k = 0; k < B.d; ++k)
            for (int i = 0; i < B.d; ++i) KA[kpos(s2.A, i, k)] = HS[(int64_t)k * B.d + i];
        int kbase = cdiv(B.d, 16) * 16;
        for (int ei : P.into[bi]) {
            const Edge& ed = P.edges[ei];
            const auto& Bs = P.blocks[ed.src];
            const auto& t = P.terms[ed.term];
            const double c = t.coef * (t.fermionic ? P.S.parity(Bs.p) : 1);
            for (int k = 0; k < Bs.d; ++k)
                for (int i = 0; i < B.d; ++i) KA[kpos(s2.A, i, kbase + k)] = c * ed.a.at(i, k);
            kbase += cdiv(Bs.d, 16) * 16;
        }
    }
}

}  // namespace dmrg
