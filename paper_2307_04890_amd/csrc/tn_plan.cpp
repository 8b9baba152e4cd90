// Host planner: turns a time-ordered event list into a level schedule of
// row-OR items for the reverse-time component matrix (Sec. 3.4).
//
// Reverse time, strict ties (Sec. 2.1): events of one time step are not
// adjacent, so every row touched at a time step must be updated from the
// rows as they were before that step.  The events of a step split into
// connected components over their nodes:
//   * a component of two nodes is a pair item: one row OR (both rows for an
//     undirected or two-way pair, only the source row for a one-way directed
//     pair, since event (u -> v) gives u's out-component everything v reaches
//     later);
//   * a component of three or more nodes is a compound item: each node x
//     gets the OR of its own row and its partners' old rows, so all of them
//     are read before any is written (gathers through scratch rows).
// Row ORs on disjoint rows commute, so each item is placed on the earliest
// level after the last level that touched any of its rows; the items of a
// level then touch pairwise disjoint rows and run concurrently.
#include <algorithm>
#include <chrono>
#include <cstring>

#include "tn_internal.h"

namespace tn {

namespace {

struct Planner {
    uint32_t n;
    bool directed;
    bool ops_mode;               // emit binary ops instead of pairs + gathers
    std::vector<uint32_t> last;  // gather form: last level (1-based) that touched a row
    uint32_t L = 0;

    // ops form: last level that wrote / read each row and scratch row
    std::vector<uint32_t> lw, lr, slw, slr;
    uint32_t S = 0, next_scratch = 0;
    struct Op {
        uint32_t a, b, d1, d2;
    };
    std::vector<Op> ops;          // ops form, in reverse-stream order
    std::vector<uint32_t> olev;   // their levels (1-based)
    int64_t n_pairs = 0, n_dir = 0, n_targets = 0, n_sources = 0;

    // items in reverse-stream order
    std::vector<uint32_t> pu, pv, plev;
    struct Gather {
        uint32_t level, tgt, s0, s1;
    };
    std::vector<Gather> gtmp;
    std::vector<uint32_t> gsrc;
    int64_t compound_items = 0;

    // per-group scratch
    std::vector<uint32_t> stamp, local;
    uint32_t gid = 0;
    std::vector<uint32_t> lnode, parent, comp, comp_nodes_ptr, comp_nodes,
        comp_ev_ptr, comp_ev, fill, nbr_ptr, nbr;
    std::vector<uint32_t> es, ed;  // group events without self-loops
    std::vector<uint32_t> posbuf;
    std::vector<uint32_t> tgt, tscr;

    Planner(uint32_t n_, bool dir, bool ops)
        : n(n_), directed(dir), ops_mode(ops), stamp(n_, 0xffffffffu), local(n_, 0) {
        if (ops) {
            lw.assign(n_, 0);
            lr.assign(n_, 0);
            grow_scratch(kOpsScratchRows);
        } else {
            last.assign(n_, 0);
        }
    }

    void grow_scratch(uint32_t rows) {
        if (rows <= S) return;
        S = rows;
        slw.resize(S, 0);
        slr.resize(S, 0);
    }
    uint32_t &W(uint32_t id) { return (id & kScratchBit) ? slw[id & kNodeMask] : lw[id]; }
    uint32_t &R(uint32_t id) { return (id & kScratchBit) ? slr[id & kNodeMask] : lr[id]; }

    // Places one op r = row[a] | row[b] -> row[d1], row[d2] (d2 may be
    // kNoRow) on the earliest level after the last write of every row it
    // reads and after the last read or write of every row it writes.
    void emit(uint32_t a, uint32_t b, uint32_t d1, uint32_t d2) {
        uint32_t lev = std::max(W(a), W(b));
        lev = std::max(lev, std::max(W(d1), R(d1)));
        if (d2 != kNoRow) lev = std::max(lev, std::max(W(d2), R(d2)));
        ++lev;
        R(a) = std::max(R(a), lev);
        R(b) = std::max(R(b), lev);
        W(d1) = lev;
        if (d2 != kNoRow) W(d2) = lev;
        if (lev > L) L = lev;
        ops.push_back({a, b, d1, d2});
        olev.push_back(lev);
    }
    // emit() for a pair of real rows: (u, v, u, v) or (u, v, u, -)
    void emit_pair(uint32_t u, uint32_t v, bool both) {
        uint32_t lev = std::max(std::max(lw[u], lr[u]), std::max(lw[v], both ? lr[v] : 0u)) + 1;
        lw[u] = lev;
        lr[u] = std::max(lr[u], lev);
        if (both) lw[v] = lev;
        lr[v] = std::max(lr[v], lev);
        if (lev > L) L = lev;
        ops.push_back({u, v, u, both ? v : kNoRow});
        olev.push_back(lev);
    }

    uint32_t find(uint32_t x) {
        while (parent[x] != x) {
            parent[x] = parent[parent[x]];
            x = parent[x];
        }
        return x;
    }

    void add_pair(uint32_t u, uint32_t v, bool uv, bool vu) {
        // uv: information reaches u's row from v (event u -> v in reverse time)
        if (ops_mode) {
            ++n_pairs;
            if (!directed || (uv && vu)) {
                emit_pair(u, v, true);
            } else {
                ++n_dir;
                if (uv) emit_pair(u, v, false);
                else emit_pair(v, u, false);
            }
            return;
        }
        uint32_t lvl = 1 + std::max(last[u], last[v]);
        last[u] = last[v] = lvl;
        if (lvl > L) L = lvl;
        if (!directed || (uv && vu)) {
            pu.push_back(u);
            pv.push_back(v);
        } else if (uv) {
            pu.push_back(u);
            pv.push_back(v | kDirBit);
        } else {
            pu.push_back(v);
            pv.push_back(u | kDirBit);
        }
        plev.push_back(lvl);
    }

    // events [a, b) share one time step (or a == b - 1 in sequential mode);
    // node ids pass through `map` when it is given (hashed networks)
    void group(const uint32_t *src, const uint32_t *dst, const uint32_t *map, int64_t a,
               int64_t b) {
        es.clear();
        ed.clear();
        for (int64_t e = a; e < b; ++e) {
            const uint32_t x = map ? map[src[e]] : src[e];
            const uint32_t y = map ? map[dst[e]] : dst[e];
            if (x != y) {
                es.push_back(x);
                ed.push_back(y);
            }
        }
        const size_t k = es.size();
        if (k == 0) return;
        if (k == 1) {
            add_pair(es[0], ed[0], true, false);
            return;
        }
        ++gid;
        if (gid == 0xffffffffu) {  // stamp wrap: reset
            std::fill(stamp.begin(), stamp.end(), 0xffffffffu);
            gid = 0;
        }
        // common case: no node occurs twice, so every event is its own pair
        // component (the stamps are then reused by the general path below)
        {
            bool disjoint = true;
            for (size_t i = 0; i < k && disjoint; ++i) {
                disjoint = stamp[es[i]] != gid && stamp[ed[i]] != gid;
                stamp[es[i]] = stamp[ed[i]] = gid;
            }
            if (disjoint) {
                for (size_t i = 0; i < k; ++i) add_pair(es[i], ed[i], true, false);
                return;
            }
            ++gid;
            if (gid == 0xffffffffu) {
                std::fill(stamp.begin(), stamp.end(), 0xffffffffu);
                gid = 0;
            }
        }
        lnode.clear();
        parent.clear();
        auto lid = [&](uint32_t x) {
            if (stamp[x] != gid) {
                stamp[x] = gid;
                local[x] = (uint32_t)lnode.size();
                lnode.push_back(x);
                parent.push_back(local[x]);
            }
            return local[x];
        };
        for (size_t i = 0; i < k; ++i) {
            uint32_t ra = find(lid(es[i])), rb = find(lid(ed[i]));
            if (ra != rb) parent[ra] = rb;
        }
        const uint32_t nl = (uint32_t)lnode.size();
        // component ids 0..nc-1 in order of first node
        comp.assign(nl, 0xffffffffu);
        std::vector<uint32_t> &root_id = fill;
        root_id.assign(nl, 0xffffffffu);
        uint32_t nc = 0;
        for (uint32_t i = 0; i < nl; ++i) {
            uint32_t r = find(i);
            if (root_id[r] == 0xffffffffu) root_id[r] = nc++;
            comp[i] = root_id[r];
        }
        // nodes per component (CSR)
        comp_nodes_ptr.assign(nc + 1, 0);
        for (uint32_t i = 0; i < nl; ++i) comp_nodes_ptr[comp[i] + 1]++;
        for (uint32_t c = 0; c < nc; ++c) comp_nodes_ptr[c + 1] += comp_nodes_ptr[c];
        comp_nodes.resize(nl);
        {
            std::vector<uint32_t> &pos = posbuf;
            pos.assign(comp_nodes_ptr.begin(), comp_nodes_ptr.end() - 1);
            for (uint32_t i = 0; i < nl; ++i) comp_nodes[pos[comp[i]]++] = i;
        }
        // events per component (CSR)
        comp_ev_ptr.assign(nc + 1, 0);
        for (size_t i = 0; i < k; ++i) comp_ev_ptr[comp[local[es[i]]] + 1]++;
        for (uint32_t c = 0; c < nc; ++c) comp_ev_ptr[c + 1] += comp_ev_ptr[c];
        comp_ev.resize(k);
        {
            std::vector<uint32_t> &pos = posbuf;
            pos.assign(comp_ev_ptr.begin(), comp_ev_ptr.end() - 1);
            for (size_t i = 0; i < k; ++i) comp_ev[pos[comp[local[es[i]]]]++] = (uint32_t)i;
        }
        for (uint32_t c = 0; c < nc; ++c) {
            const uint32_t n0 = comp_nodes_ptr[c], n1 = comp_nodes_ptr[c + 1];
            const uint32_t e0 = comp_ev_ptr[c], e1 = comp_ev_ptr[c + 1];
            if (n1 - n0 == 2) {
                uint32_t x = lnode[comp_nodes[n0]], y = lnode[comp_nodes[n0 + 1]];
                bool xy = false, yx = false;
                for (uint32_t q = e0; q < e1; ++q) {
                    uint32_t i = comp_ev[q];
                    if (es[i] == x) xy = true; else yx = true;
                }
                add_pair(x, y, xy, yx);
                continue;
            }
            compound(n0, n1, e0, e1);
        }
    }

    // partners of each node of a compound item: event s -> d gives
    // new[s] |= old[d] (and new[d] |= old[s] when undirected); fills nbr /
    // nbr_ptr indexed by the node's position in the item
    void partners(uint32_t n0, uint32_t n1, uint32_t e0, uint32_t e1) {
        const uint32_t cn = n1 - n0;
        for (uint32_t q = n0; q < n1; ++q) fill[comp_nodes[q]] = q - n0;
        nbr_ptr.assign(cn + 1, 0);
        for (uint32_t q = e0; q < e1; ++q) {
            uint32_t i = comp_ev[q];
            nbr_ptr[fill[local[es[i]]] + 1]++;
            if (!directed) nbr_ptr[fill[local[ed[i]]] + 1]++;
        }
        for (uint32_t c = 0; c < cn; ++c) nbr_ptr[c + 1] += nbr_ptr[c];
        nbr.resize(nbr_ptr[cn]);
        std::vector<uint32_t> &pos = posbuf;
        pos.assign(nbr_ptr.begin(), nbr_ptr.end() - 1);
        for (uint32_t q = e0; q < e1; ++q) {
            uint32_t i = comp_ev[q];
            nbr[pos[fill[local[es[i]]]]++] = ed[i];
            if (!directed) nbr[pos[fill[local[ed[i]]]]++] = es[i];
        }
        for (uint32_t c = 0; c < cn; ++c) std::sort(nbr.begin() + nbr_ptr[c], nbr.begin() + nbr_ptr[c + 1]);
    }

    // Compound item as binary ops: each target folds its old row and its
    // partners' old rows into a scratch row (all folds read only old rows),
    // then every target copies its scratch row back.  A compound of more
    // targets than the default scratch folds its last target into its own
    // row instead: emit() places those in-place ops after every other fold
    // that reads the old row, and the partners' rows they read are only
    // written by the copies back, which come later.  Such an item then needs
    // targets - 1 scratch rows, so a network of K nodes never needs more
    // than K - 1.
    void compound_ops(uint32_t n0, uint32_t n1, uint32_t e0, uint32_t e1) {
        partners(n0, n1, e0, e1);
        const uint32_t cn = n1 - n0;
        uint32_t targets = 0;
        for (uint32_t c = 0; c < cn; ++c) {
            const uint32_t x = lnode[comp_nodes[n0 + c]];
            for (uint32_t q = nbr_ptr[c]; q < nbr_ptr[c + 1]; ++q)
                if (nbr[q] != x) {
                    ++targets;
                    break;
                }
        }
        if (targets == 0) return;
        const bool in_place = targets > kOpsScratchRows;
        grow_scratch(in_place ? targets - 1 : targets);
        tgt.clear();
        tscr.clear();
        uint32_t seen = 0;
        for (uint32_t c = 0; c < cn; ++c) {
            const uint32_t b0 = nbr_ptr[c], b1 = nbr_ptr[c + 1];
            const uint32_t x = lnode[comp_nodes[n0 + c]];
            bool has = false;
            for (uint32_t q = b0; q < b1 && !has; ++q) has = nbr[q] != x;
            if (!has) continue;  // no incoming information: row unchanged
            const bool own = in_place && ++seen == targets;
            const uint32_t tsc = own ? x : ((next_scratch++ % S) | kScratchBit);
            uint32_t acc = x;
            int64_t k = 0;
            for (uint32_t q = b0; q < b1; ++q) {
                if ((q > b0 && nbr[q] == nbr[q - 1]) || nbr[q] == x) continue;
                emit(acc, nbr[q], tsc, kNoRow);
                acc = tsc;
                ++k;
            }
            ++n_targets;
            n_sources += k + 1;
            if (own) continue;
            tgt.push_back(x);
            tscr.push_back(tsc);
        }
        for (size_t i = 0; i < tgt.size(); ++i) emit(tscr[i], tscr[i], tgt[i], kNoRow);
    }

    void compound(uint32_t n0, uint32_t n1, uint32_t e0, uint32_t e1) {
        ++compound_items;
        if (ops_mode) {
            compound_ops(n0, n1, e0, e1);
            return;
        }
        uint32_t lvl = 0;
        for (uint32_t q = n0; q < n1; ++q) lvl = std::max(lvl, last[lnode[comp_nodes[q]]]);
        ++lvl;
        if (lvl > L) L = lvl;
        for (uint32_t q = n0; q < n1; ++q) last[lnode[comp_nodes[q]]] = lvl;
        partners(n0, n1, e0, e1);
        const uint32_t cn = n1 - n0;
        for (uint32_t c = 0; c < cn; ++c) {
            uint32_t b0 = nbr_ptr[c], b1 = nbr_ptr[c + 1];
            if (b0 == b1) continue;  // no incoming information: row unchanged
            uint32_t x = lnode[comp_nodes[n0 + c]];
            Gather g;
            g.level = lvl;
            g.tgt = x;
            g.s0 = (uint32_t)gsrc.size();
            gsrc.push_back(x);
            for (uint32_t q = b0; q < b1; ++q)
                if (q == b0 || nbr[q] != nbr[q - 1])
                    if (nbr[q] != x) gsrc.push_back(nbr[q]);
            g.s1 = (uint32_t)gsrc.size();
            gtmp.push_back(g);
        }
    }
};

}  // namespace

namespace {

// Binary-op form: levels of at most kOpsLevelCap ops (a wider level is split
// into consecutive levels; its ops are independent, so any split is exact).
void finish_ops(Planner &p, HostSchedule &out) {
    const uint32_t L = p.L;
    const size_t P = p.ops.size();
    std::vector<uint32_t> cnt((size_t)L + 1, 0);
    for (uint32_t lv : p.olev) cnt[lv]++;
    std::vector<uint32_t> base((size_t)L + 2, 0);  // first split level of level l
    for (uint32_t l = 1; l <= L; ++l)
        base[l + 1] = base[l] + std::max<uint32_t>(1, (cnt[l] + kOpsLevelCap - 1) / kOpsLevelCap);
    const uint32_t Lf = base[L + 1];
    out.Lops = Lf;
    out.lvl_op.assign((size_t)Lf + 1, 0);
    out.ops.resize(4 * P);
    if (Lf == L) {
        // no level is split (the usual case): one counting-sort pass
        for (uint32_t l = 0; l < L; ++l) out.lvl_op[l + 1] = out.lvl_op[l] + cnt[l + 1];
        std::vector<uint32_t> pos(out.lvl_op.begin(), out.lvl_op.end() - 1);
        for (size_t i = 0; i < P; ++i) {
            const size_t q = pos[p.olev[i] - 1]++;
            std::memcpy(&out.ops[4 * q], &p.ops[i], sizeof(Planner::Op));
        }
    } else {
        std::vector<uint32_t> fcnt(Lf, 0), rank((size_t)L + 1, 0), flev(P);
        for (size_t i = 0; i < P; ++i) {
            const uint32_t lv = p.olev[i];
            flev[i] = base[lv] + rank[lv]++ / kOpsLevelCap;
            fcnt[flev[i]]++;
        }
        for (uint32_t l = 0; l < Lf; ++l) out.lvl_op[l + 1] = out.lvl_op[l] + fcnt[l];
        std::vector<uint32_t> pos(out.lvl_op.begin(), out.lvl_op.end() - 1);
        for (size_t i = 0; i < P; ++i) {
            const size_t q = pos[flev[i]]++;
            std::memcpy(&out.ops[4 * q], &p.ops[i], sizeof(Planner::Op));
        }
    }
    out.scratch_rows = p.S;
    out.op_levels_unsplit = L;
}

}  // namespace

tn_status plan_events(uint32_t n, int64_t m, const uint32_t *src,
                      const uint32_t *dst, const int64_t *t, uint32_t flags,
                      HostSchedule &out, std::string &err, const uint32_t *map,
                      uint32_t n_src, int forms) {
    auto t0 = std::chrono::steady_clock::now();
    if (n == 0) { err = "n must be > 0"; return TN_E_ARG; }
    if (m < 0) { err = "m must be >= 0"; return TN_E_ARG; }
    if (m > 0 && (!src || !dst || !t)) { err = "null event array"; return TN_E_ARG; }
    if (flags & ~(uint32_t)(TN_DIRECTED | TN_TIES_SEQUENTIAL | TN_FORWARD)) { err = "unknown flag bits"; return TN_E_ARG; }
    if (n > kNodeMask) { err = "n must be < 2^31"; return TN_E_UNSUPPORTED; }
    if (m >= (int64_t)0xffffffffLL) { err = "m must be < 2^32 - 1"; return TN_E_UNSUPPORTED; }
    const uint32_t id_limit = map ? n_src : n;
    if (map)
        for (uint32_t x = 0; x < n_src; ++x)
            if (map[x] >= n) {
                err = "node map sends node " + std::to_string(x) + " past the last super-node";
                return TN_E_RANGE;
            }
    for (int64_t e = 0; e < m; ++e) {
        if (src[e] >= id_limit || dst[e] >= id_limit) {
            err = "event " + std::to_string(e) + " has a node id >= n";
            return TN_E_RANGE;
        }
        if (e > 0 && t[e] < t[e - 1]) {
            err = "event " + std::to_string(e) + " is earlier than its predecessor";
            return TN_E_ORDER;
        }
    }
    const bool directed = flags & TN_DIRECTED;
    const bool seq = flags & TN_TIES_SEQUENTIAL;
    out.n = n;
    out.m = m;
    out.flags = flags;
    // Reverse time: time steps from the last, an event (u, v) brings v's row
    // into u's.  Forward time (Algorithm 1 as printed): time steps from the
    // first, and (u, v) brings u's row into v's, i.e. the reverse-time rule
    // applied to (v, u).
    const bool forward = flags & TN_FORWARD;
    auto walk = [&](Planner &pl) {
        if (forward) {
            int64_t a = 0;
            while (a < m) {
                int64_t b = a + 1;
                if (!seq)
                    while (b < m && t[b] == t[a]) ++b;
                pl.group(dst, src, map, a, b);
                a = b;
            }
            return;
        }
        int64_t b = m;
        while (b > 0) {
            int64_t a = b - 1;
            if (!seq)
                while (a > 0 && t[a - 1] == t[b - 1]) --a;
            pl.group(src, dst, map, a, b);
            b = a;
        }
    };
    if (forms & kFormOps) {
        Planner po(n, directed, true);
        po.ops.reserve((size_t)m + (size_t)m / 4);
        po.olev.reserve((size_t)m + (size_t)m / 4);
        walk(po);
        finish_ops(po, out);
        out.op_pairs = po.n_pairs;
        out.op_directed = po.n_dir;
        out.op_targets = po.n_targets;
        out.op_sources = po.n_sources;
        out.op_compound = po.compound_items;
        if (!(forms & kFormGather)) {
            out.L = 0;
            out.lvl_pair.assign(1, 0);
            out.lvl_gat.assign(1, 0);
            out.compound_items = po.compound_items;
            out.directed_pairs = po.n_dir;
            out.host_seconds =
                std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
            return TN_OK;
        }
    }
    Planner p(n, directed, false);
    p.pu.reserve((size_t)m);
    p.pv.reserve((size_t)m);
    p.plev.reserve((size_t)m);
    walk(p);
    // counting sort by level
    const uint32_t L = p.L;
    out.L = L;
    out.lvl_pair.assign((size_t)L + 1, 0);
    out.lvl_gat.assign((size_t)L + 1, 0);
    for (uint32_t lv : p.plev) out.lvl_pair[lv]++;  // level lv (1-based) -> slot lv
    for (auto &g : p.gtmp) out.lvl_gat[g.level]++;
    out.max_level_items = 0;
    out.max_level_gathers = 0;
    for (uint32_t l = 1; l <= L; ++l) {
        int64_t w = (int64_t)out.lvl_pair[l] + out.lvl_gat[l];
        out.max_level_items = std::max(out.max_level_items, w);
        out.max_level_gathers = std::max<int64_t>(out.max_level_gathers, out.lvl_gat[l]);
    }
    for (uint32_t l = 0; l < L; ++l) {
        out.lvl_pair[l + 1] += out.lvl_pair[l];
        out.lvl_gat[l + 1] += out.lvl_gat[l];
    }
    const size_t P = p.pu.size();
    out.pairs.resize(2 * P);
    {
        std::vector<uint32_t> pos(out.lvl_pair.begin(), out.lvl_pair.end() - 1);
        for (size_t i = 0; i < P; ++i) {
            uint32_t q = pos[p.plev[i] - 1]++;
            out.pairs[2 * (size_t)q] = p.pu[i];
            out.pairs[2 * (size_t)q + 1] = p.pv[i];
        }
    }
    const size_t G = p.gtmp.size();
    out.gat_tgt.resize(G);
    out.gat_ptr.assign(G + 1, 0);
    out.gat_src.resize(p.gsrc.size());
    {
        std::vector<uint32_t> order(G);
        std::vector<uint32_t> pos(out.lvl_gat.begin(), out.lvl_gat.end() - 1);
        for (size_t i = 0; i < G; ++i) order[pos[p.gtmp[i].level - 1]++] = (uint32_t)i;
        uint32_t s = 0;
        for (size_t q = 0; q < G; ++q) {
            const auto &g = p.gtmp[order[q]];
            out.gat_tgt[q] = g.tgt;
            out.gat_ptr[q] = s;
            for (uint32_t r = g.s0; r < g.s1; ++r) out.gat_src[s++] = p.gsrc[r];
        }
        out.gat_ptr[G] = s;
    }
    out.compound_items = p.compound_items;
    out.directed_pairs = 0;
    for (size_t i = 0; i < P; ++i) out.directed_pairs += (p.pv[i] & kDirBit) ? 1 : 0;
    out.host_seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    return TN_OK;
}

namespace {
inline size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

struct Layout {
    size_t lvl_pair, lvl_gat, pairs, gat_tgt, gat_ptr, gat_src, total;
};

Layout layout_of(const HostSchedule &s) {
    Layout o;
    size_t off = 0;
    o.lvl_pair = off; off = align256(off + 4 * s.lvl_pair.size());
    o.lvl_gat = off;  off = align256(off + 4 * s.lvl_gat.size());
    o.pairs = off;    off = align256(off + 4 * s.pairs.size());
    o.gat_tgt = off;  off = align256(off + 4 * s.gat_tgt.size());
    o.gat_ptr = off;  off = align256(off + 4 * s.gat_ptr.size());
    o.gat_src = off;  off = align256(off + 4 * s.gat_src.size());
    o.total = std::max<size_t>(off, 256);
    return o;
}
}  // namespace

size_t schedule_device_bytes(const HostSchedule &s) { return layout_of(s).total; }

void schedule_pieces(const HostSchedule &s, std::vector<SchedPiece> &out) {
    const Layout o = layout_of(s);
    out.clear();
    auto put = [&](size_t off, const std::vector<uint32_t> &v) {
        if (!v.empty()) out.push_back({off, v.data(), 4 * v.size()});
    };
    put(o.lvl_pair, s.lvl_pair);
    put(o.lvl_gat, s.lvl_gat);
    put(o.pairs, s.pairs);
    put(o.gat_tgt, s.gat_tgt);
    put(o.gat_ptr, s.gat_ptr);
    put(o.gat_src, s.gat_src);
}

size_t ops_device_bytes(const HostSchedule &s) {
    return align256(4 * s.lvl_op.size()) + align256(4 * std::max<size_t>(s.ops.size(), 4));
}

void ops_pack(const HostSchedule &s, std::vector<unsigned char> &img) {
    img.assign(ops_device_bytes(s), 0);
    std::memcpy(img.data(), s.lvl_op.data(), 4 * s.lvl_op.size());
    if (!s.ops.empty())
        std::memcpy(img.data() + align256(4 * s.lvl_op.size()), s.ops.data(), 4 * s.ops.size());
}

DevOps ops_view(const HostSchedule &s, const void *dev_base) {
    const unsigned char *b = (const unsigned char *)dev_base;
    DevOps d;
    d.L = s.Lops;
    d.nops = (uint32_t)(s.ops.size() / 4);
    d.lvl = (const uint32_t *)b;
    d.ops = (const uint4 *)(b + align256(4 * s.lvl_op.size()));
    return d;
}

void schedule_pack(const HostSchedule &s, std::vector<unsigned char> &img) {
    Layout o = layout_of(s);
    img.assign(o.total, 0);
    auto put = [&](size_t off, const std::vector<uint32_t> &v) {
        if (!v.empty()) std::memcpy(img.data() + off, v.data(), 4 * v.size());
    };
    put(o.lvl_pair, s.lvl_pair);
    put(o.lvl_gat, s.lvl_gat);
    put(o.pairs, s.pairs);
    put(o.gat_tgt, s.gat_tgt);
    put(o.gat_ptr, s.gat_ptr);
    put(o.gat_src, s.gat_src);
}

DevSchedule schedule_view(const HostSchedule &s, const void *dev_base) {
    Layout o = layout_of(s);
    const unsigned char *b = (const unsigned char *)dev_base;
    DevSchedule d;
    d.n = s.n;
    d.L = s.L;
    d.max_gat = (uint32_t)s.max_level_gathers;
    d.pad_ = 0;
    d.lvl_pair = (const uint32_t *)(b + o.lvl_pair);
    d.lvl_gat = (const uint32_t *)(b + o.lvl_gat);
    d.pairs = (const uint2 *)(b + o.pairs);
    d.gat_tgt = (const uint32_t *)(b + o.gat_tgt);
    d.gat_ptr = (const uint32_t *)(b + o.gat_ptr);
    d.gat_src = (const uint32_t *)(b + o.gat_src);
    return d;
}

}  // namespace tn

namespace tn {

// The forwarded form of an op schedule (see tn_internal.h).  Levels wider
// than kFwdLevelCap are cut into consecutive parts of near-equal size (the
// ops of a level are independent, so any split keeps the result).  A forward
// pass then rewrites every operand last written by the level just before
// as that writer's index in it (kFwdHot); a backward pass flags every
// destination whose row the next level overwrites (kFwdNoStore): that
// level reads the row, if at all, from the forwarded copy, so memory never
// needs the value.  Rows are keyed n + id for scratch rows.
void fwd_schedule(const std::vector<uint32_t> &lvl_op, const std::vector<uint32_t> &ops,
                  uint32_t n, uint32_t scratch_rows, uint32_t cap, std::vector<uint32_t> &flvl,
                  std::vector<uint32_t> &fops) {
    if (cap == 0 || cap > kFwdLevelCap) cap = kFwdLevelCap;
    const uint32_t Lops = lvl_op.empty() ? 0 : (uint32_t)lvl_op.size() - 1;
    const size_t keys = (size_t)n + scratch_rows + 1;
    auto key = [n](uint32_t id) -> size_t {
        return (id & kScratchBit) ? (size_t)n + (id & kNodeMask) : (size_t)id;
    };
    flvl.assign(1, 0);
    fops.clear();
    fops.reserve(ops.size());
    // the ops in their new order, without the forwarding bits
    std::vector<uint32_t> rops;
    rops.reserve(ops.size());
    // forward: the level and index of each row's last write
    std::vector<uint32_t> wl(keys, 0xffffffffu), wj(keys, 0);
    std::vector<uint32_t> rest, next, both, other;
    uint32_t L = 0;  // forwarded levels so far
    for (uint32_t l = 0; l < Lops; ++l) {
        rest.clear();
        for (uint32_t q = lvl_op[l]; q < lvl_op[l + 1]; ++q) rest.push_back(q);
        // an op level becomes parts of at most cap ops, of even size; an
        // operand is forwarded iff its row was written by the part just
        // before, so it is decided part by part (ops of one op level touch
        // disjoint rows)
        while (!rest.empty()) {
            const size_t parts = (rest.size() + cap - 1) / cap;
            const size_t target = (rest.size() + parts - 1) / parts;
            auto hot = [&](uint32_t id) { return L > 0 && wl[key(id)] == L - 1; };
            both.clear();
            other.clear();
            next.clear();
            for (uint32_t q : rest) {
                const bool cold2 = !hot(ops[4 * (size_t)q]) && !hot(ops[4 * (size_t)q + 1]);
                if (both.size() + other.size() >= target)
                    next.push_back(q);
                else
                    (cold2 ? both : other).push_back(q);
            }
            const uint32_t base = (uint32_t)(rops.size() / 4);
            uint32_t j = 0;
            for (const std::vector<uint32_t> *grp : {&both, &other})
                for (uint32_t q : *grp) {
                    uint32_t x = ops[4 * (size_t)q], y = ops[4 * (size_t)q + 1];
                    if (!hot(x) && hot(y)) std::swap(x, y);  // the one from memory goes second
                    const uint32_t d1 = ops[4 * (size_t)q + 2], d2 = ops[4 * (size_t)q + 3];
                    rops.insert(rops.end(), {x, y, d1, d2});
                    fops.insert(fops.end(), {hot(x) ? kFwdHot | wj[key(x)] : x,
                                             hot(y) ? kFwdHot | wj[key(y)] : y, d1, d2});
                    ++j;
                }
            for (uint32_t q = base; q < base + j; ++q)
                for (int i = 2; i < 4; ++i) {
                    const uint32_t d = rops[4 * (size_t)q + i];
                    if (d == kNoRow) continue;
                    wl[key(d)] = L;
                    wj[key(d)] = q - base;
                }
            flvl.push_back(base + j);
            ++L;
            rest.swap(next);
        }
    }
    // backward: the level of each row's next write
    std::fill(wl.begin(), wl.end(), 0xffffffffu);
    for (uint32_t l = L; l-- > 0;) {
        const uint32_t q0 = flvl[l], q1 = flvl[l + 1];
        for (uint32_t q = q0; q < q1; ++q)
            for (int i = 2; i < 4; ++i) {
                const uint32_t d = rops[4 * (size_t)q + i];
                if (d == kNoRow) continue;
                if (wl[key(d)] == l + 1) fops[4 * (size_t)q + i] = d | kFwdNoStore;
            }
        for (uint32_t q = q0; q < q1; ++q)
            for (int i = 2; i < 4; ++i) {
                const uint32_t d = rops[4 * (size_t)q + i];
                if (d != kNoRow) wl[key(d)] = l;
            }
    }
}

}  // namespace tn
