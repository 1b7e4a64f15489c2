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

// Block of an operator (or its transpose) leaving sector src.  Returns the destination sector
// or -1; M(i, j) = element (i, j) of the (dst x src) block.
struct OpRef {
    int dst = -1;
    const double* data = nullptr;
    int ld = 0;         // leading dimension of the stored block
    bool transposed = false;
    double at(int i, int j) const { return transposed ? data[(int64_t)i * ld + j] : data[(int64_t)j * ld + i]; }
};

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

// Offset of element (i, k) inside a packed factor: i = row (stage 2) or column (stage 1),
// k = K index counted from the start of the packed K range, nch = K chunks per panel.
int64_t packed_index(int i, int k, int nch) {
    const int pnl = i / kPanel, r = i % kPanel;
    const int ch = k / kChunk, g = (k % kChunk) / 4, t = k % 4;
    return (((int64_t)pnl * nch + ch) * 4 + g) * (kPanel * 4) + r * 4 + t;
}

// Reorders a tile list (tiles of one block contiguous) for launch: work groups of `group`
// consecutive tiles, work group i runs on XCD i mod kXcd.  Blocks are assigned to XCDs by
// longest-processing-time on their weights; per XCD the blocks are ordered heaviest first;
// the per-XCD lists are padded with empty tiles (blk = -1) to whole groups and equal length.
std::vector<Tile> xcd_order(const std::vector<Tile>& tiles, const std::vector<double>& w,
                            int group) {
    const int nb = (int)w.size();
    std::vector<std::vector<Tile>> of(nb);
    for (const Tile& t : tiles) of[t.blk].push_back(t);
    std::vector<int> order(nb);
    for (int i = 0; i < nb; ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return w[a] > w[b]; });
    std::vector<double> load(kXcd, 0.0);
    std::vector<std::vector<Tile>> lists(kXcd);
    for (int bi : order) {
        if (of[bi].empty()) continue;
        int x = 0;
        for (int i = 1; i < kXcd; ++i)
            if (load[i] < load[x]) x = i;
        load[x] += w[bi];
        lists[x].insert(lists[x].end(), of[bi].begin(), of[bi].end());
    }
    size_t groups = 0;
    for (auto& l : lists) {
        while (l.size() % group) l.push_back(Tile{-1, 0, 0, 0});
        groups = std::max(groups, l.size() / group);
    }
    for (auto& l : lists)
        while (l.size() < groups * group) l.push_back(Tile{-1, 0, 0, 0});
    std::vector<Tile> out;
    out.reserve(groups * group * kXcd);
    for (size_t gi = 0; gi < groups; ++gi)
        for (int x = 0; x < kXcd; ++x)
            out.insert(out.end(), lists[x].begin() + gi * group, lists[x].begin() + (gi + 1) * group);
    return out;
}

void tile_list(std::vector<Tile>& out, int blk, int M, int N, int tm, int tn) {
    for (int m0 = 0; m0 < M; m0 += tm)
        for (int n0 = 0; n0 < N; n0 += tn) out.push_back(Tile{blk, m0, n0, 0});
}

}  // namespace

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

    // outgoing terms per source block
    struct Edge {
        int src, dst, term;
        OpRef a, b;
        int col;          // first column of the right factor inside R_src
    };
    std::vector<Edge> edges;
    std::vector<std::vector<int>> out_of(nb), into(nb);
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
            edges.push_back(Edge{bi, dst, (int)ti, a, b, 0});
            out_of[bi].push_back((int)edges.size() - 1);
            into[dst].push_back((int)edges.size() - 1);
        }
    }

    // stage 1: R_b = [H_E(q)^T | B_1^T | ...], T_b = X_b R_b
    double flops = 0.0;
    int64_t toff = 0;
    for (int bi = 0; bi < nb; ++bi) {
        const auto& B = P.blocks[bi];
        int N = B.e;
        for (int ei : out_of[bi]) {
            edges[ei].col = N;
            N += P.blocks[edges[ei].dst].e;
        }
        S1Block s;
        s.M = 2 * B.d;
        s.K = B.e;
        s.N = N;
        s.prob = 0;
        s.nch = (B.e + kChunk - 1) / kChunk;
        s.pad = 0;
        s.X = View{B.off, P.n, B.d, B.d};
        s.Roff = (int64_t)P.R.size();
        const int dpad = round_up(B.d, 4);
        s.T = View{toff, dpad, 2 * dpad, B.d};
        toff += (int64_t)2 * dpad * N;
        // pack R (K x N) by column panels, zero padding to whole tiles and chunks
        const int Npad = round_up(N, kTile1N);
        P.R.resize(P.R.size() + (size_t)Npad * s.nch * kChunk, 0.0);
        double* R = P.R.data() + s.Roff;
        const double* HE = P.E.H.data() + P.E.hoff[B.q];
        for (int j = 0; j < B.e; ++j)          // R(k, j) = H_E(q)(j, k)
            for (int k = 0; k < B.e; ++k) R[packed_index(j, k, s.nch)] = HE[(int64_t)k * B.e + j];
        for (int ei : out_of[bi]) {
            const Edge& ed = edges[ei];
            const int e2 = P.blocks[ed.dst].e;
            for (int j = 0; j < e2; ++j)          // R(k, col + j) = B(j, k)
                for (int k = 0; k < B.e; ++k)
                    R[packed_index(ed.col + j, k, s.nch)] = ed.b.at(j, k);
        }
        flops += 2.0 * s.M * (double)s.K * s.N;
        P.flops1 += 2.0 * s.M * (double)s.K * s.N;
        P.s1.push_back(s);
        tile_list(P.tiles1, bi, s.M, s.N, kTile, kTile1N);
    }
    P.T_size = toff;

    // stage 2: Y_b' = T0 + [H_S(p') | s A ...] [X_b' ; T parts]
    for (int bi = 0; bi < nb; ++bi) {
        const auto& B = P.blocks[bi];
        S2Block s;
        s.M = B.d;
        s.N = 2 * B.e;
        s.prob = 0;
        s.seg0 = (int)P.segs.size();
        s.Aoff = (int64_t)P.A.size();
        s.T0 = View{P.s1[bi].T.off, P.s1[bi].T.poff, P.s1[bi].T.ld, B.e};
        s.Y = View{B.off, P.n, B.d, B.e};
        int kA = 0, nch = 0;
        // diagonal H_S term on the block itself
        Segment g0;
        g0.K = B.d;
        g0.ch0 = 0;
        g0.src = 0;
        g0.pad = 0;
        g0.B = View{B.off, P.n, B.d, B.e};
        P.segs.push_back(g0);
        kA += B.d;
        nch += (B.d + kChunk - 1) / kChunk;
        for (int ei : into[bi]) {
            const Edge& ed = edges[ei];
            const auto& Bs = P.blocks[ed.src];
            Segment g;
            g.K = Bs.d;
            g.ch0 = nch;
            g.src = 1;
            g.pad = 0;
            const View& ts = P.s1[ed.src].T;
            g.B = View{ts.off + (int64_t)ed.col * ts.ld, ts.poff, ts.ld, B.e};
            P.segs.push_back(g);
            kA += Bs.d;
            nch += (Bs.d + kChunk - 1) / kChunk;
        }
        s.nseg = (int)P.segs.size() - s.seg0;
        s.nch = nch;
        // pack Acat (d' x Kcat) by row panels, each segment starting on a fresh chunk
        const int Mpad = round_up(B.d, kTile);
        P.A.resize(P.A.size() + (size_t)Mpad * nch * kChunk, 0.0);
        double* A = P.A.data() + s.Aoff;
        const double* HS = P.S.H.data() + P.S.hoff[B.p];
        for (int k = 0; k < B.d; ++k)
            for (int i = 0; i < B.d; ++i) A[packed_index(i, k, nch)] = HS[(int64_t)k * B.d + i];
        int si = 1;
        for (int ei : into[bi]) {
            const Edge& ed = edges[ei];
            const auto& Bs = P.blocks[ed.src];
            const auto& t = P.terms[ed.term];
            const double c = t.coef * (t.fermionic ? P.S.parity(Bs.p) : 1);
            const int kbase = P.segs[s.seg0 + si].ch0 * kChunk;
            for (int k = 0; k < Bs.d; ++k)
                for (int i = 0; i < B.d; ++i) A[packed_index(i, kbase + k, nch)] = c * ed.a.at(i, k);
            ++si;
        }
        flops += 2.0 * s.M * (double)s.N * kA;
        P.flops2 += 2.0 * s.M * (double)s.N * kA;
        P.s2.push_back(s);
        tile_list(P.tiles2, bi, s.M, s.N, kTile, kTile);
    }
    P.flops = flops;

    // XCD-aware launch order: every block's tiles go to one XCD (so its packed factor panels
    // and source panels are shared in that XCD's L2), blocks are spread over the XCDs by
    // longest-processing-time, heaviest first inside each XCD.
    std::vector<double> w1(nb), w2(nb);
    for (int bi = 0; bi < nb; ++bi) {
        int k = 0;
        for (int s = 0; s < P.s2[bi].nseg; ++s) k += P.segs[P.s2[bi].seg0 + s].K;
        const double nt1 = (double)((P.s1[bi].M + kTile - 1) / kTile) * ((P.s1[bi].N + kTile1N - 1) / kTile1N);
        const double nt2 = (double)((P.s2[bi].M + kTile - 1) / kTile) * ((P.s2[bi].N + kTile - 1) / kTile);
        w1[bi] = nt1 * (P.s1[bi].nch + 1);
        w2[bi] = nt2 * ((k + kChunk - 1) / kChunk + 2);
    }
    P.tiles1 = xcd_order(P.tiles1, w1, kWaves);
    P.tiles2 = xcd_order(P.tiles2, w2, 1);
    return "";
}

}  // namespace dmrg
