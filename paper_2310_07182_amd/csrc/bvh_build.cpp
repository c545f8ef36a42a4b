// Host BVH2 builder: binned surface-area heuristic (64 centroid bins per axis,
// traversal and intersection cost 1), leaves of at most kMaxLeaf triangles,
// object-median splits once the remaining depth budget only just fits a
// balanced subtree, so that the leaf depth never exceeds kMaxDepth.  Large subtrees are built on separate threads; the output
// (node order, triangle order) does not depend on thread timing because every
// subtree is built from its own triangle range and the nodes are numbered by a
// final depth-first pass.
//
// The BVH only prunes: the closest hit is the (t, prim id) minimum over all
// triangles, whatever BVH is used.

#include <algorithm>
#include <atomic>
#include <cmath>
#include <array>
#include <cstring>
#include <functional>
#include <future>
#include <limits>
#include <thread>

#include "pt_internal.h"

namespace pt {
namespace {

constexpr int kBins = 64;
constexpr uint32_t kParallelMin = 1u << 16;
constexpr uint32_t kParallelBinMin = 1u << 20;

struct Box {
    float lo[3] = {INFINITY, INFINITY, INFINITY};
    float hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    void grow(const float* l, const float* h) {
        for (int a = 0; a < 3; ++a) {
            lo[a] = std::min(lo[a], l[a]);
            hi[a] = std::max(hi[a], h[a]);
        }
    }
    void grow(const Box& b) { grow(b.lo, b.hi); }
    double half_area() const {
        double dx = (double)hi[0] - lo[0], dy = (double)hi[1] - lo[1], dz = (double)hi[2] - lo[2];
        if (dx < 0 || dy < 0 || dz < 0) return 0.0;
        return dx * dy + dy * dz + dz * dx;
    }
};

struct BNode {
    Box box;
    int32_t left = -1, right = -1;   // children (build-node ids); -1 = leaf
    uint32_t first = 0, count = 0;
    uint32_t depth = 0;
};

struct Builder {
    const float* tris;
    std::vector<float> tlo, thi, cen;   // per-triangle bounds and centroid
    std::vector<uint32_t> idx;
    std::vector<BNode> nodes;
    std::atomic<uint32_t> nnodes{0};
    std::atomic<int> threads_left{0};

    uint32_t alloc() { return nnodes.fetch_add(1, std::memory_order_relaxed); }

    void bin_range(uint32_t first, uint32_t n, int axis, float clo, double scale, Box* bb, uint32_t* cnt) {
        for (uint32_t i = 0; i < n; ++i) {
            uint32_t p = idx[first + i];
            int b = (int)(((double)cen[3 * (size_t)p + axis] - clo) * scale);
            b = std::min(std::max(b, 0), kBins - 1);
            ++cnt[b];
            bb[b].grow(&tlo[3 * (size_t)p], &thi[3 * (size_t)p]);
        }
    }

    void build(uint32_t node, uint32_t first, uint32_t n, uint32_t depth) {
        BNode& nd = nodes[node];
        nd.depth = depth;
        Box cb;
        Box bb;
        for (uint32_t i = 0; i < n; ++i) {
            uint32_t p = idx[first + i];
            bb.grow(&tlo[3 * (size_t)p], &thi[3 * (size_t)p]);
            cb.grow(&cen[3 * (size_t)p], &cen[3 * (size_t)p]);
        }
        nd.box = bb;
        if (n <= (uint32_t)kMaxLeaf) {
            nd.first = first;
            nd.count = n;
            return;
        }
        uint32_t mid = 0;
        // switch to object-median splits while a balanced subtree still fits the depth budget
        uint32_t need = 0;
        for (uint64_t m = n; m > (uint64_t)kMaxLeaf; m = (m + 1) / 2) ++need;
        bool median = depth + need + 2 >= (uint32_t)kMaxDepth;
        int best_axis = -1, best_split = 0;
        if (!median) {
            double best = std::numeric_limits<double>::infinity();
            for (int a = 0; a < 3; ++a) {
                double ext = (double)cb.hi[a] - cb.lo[a];
                if (!(ext > 0.0)) continue;
                double scale = kBins / ext;
                Box bins[kBins];
                uint32_t cnt[kBins] = {0};
                if (n >= kParallelBinMin) {
                    unsigned T = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
                    std::vector<std::array<Box, kBins>> pb(T);
                    std::vector<std::array<uint32_t, kBins>> pc(T);
                    std::vector<std::thread> th;
                    uint32_t chunk = (n + T - 1) / T;
                    for (unsigned t = 0; t < T; ++t) {
                        pc[t].fill(0);
                        uint32_t f = first + t * chunk;
                        uint32_t m = std::min(chunk, first + n - std::min(f, first + n));
                        th.emplace_back([&, t, f, m] { bin_range(f, m, a, cb.lo[a], scale, pb[t].data(), pc[t].data()); });
                    }
                    for (auto& x : th) x.join();
                    for (unsigned t = 0; t < T; ++t)
                        for (int b = 0; b < kBins; ++b) {
                            bins[b].grow(pb[t][b]);
                            cnt[b] += pc[t][b];
                        }
                } else {
                    bin_range(first, n, a, cb.lo[a], scale, bins, cnt);
                }
                double rarea[kBins];
                uint32_t rcnt[kBins];
                Box r;
                uint32_t rc = 0;
                for (int b = kBins - 1; b > 0; --b) {
                    r.grow(bins[b]);
                    rc += cnt[b];
                    rarea[b] = r.half_area();
                    rcnt[b] = rc;
                }
                Box l;
                uint32_t lc = 0;
                for (int b = 0; b < kBins - 1; ++b) {
                    l.grow(bins[b]);
                    lc += cnt[b];
                    if (lc == 0 || rcnt[b + 1] == 0) continue;
                    double c = l.half_area() * lc + rarea[b + 1] * rcnt[b + 1];
                    if (c < best) {
                        best = c;
                        best_axis = a;
                        best_split = b + 1;
                    }
                }
            }
        }
        if (best_axis >= 0) {
            double scale = kBins / ((double)cb.hi[best_axis] - cb.lo[best_axis]);
            float clo = cb.lo[best_axis];
            auto it = std::partition(idx.begin() + first, idx.begin() + first + n, [&](uint32_t p) {
                int b = (int)(((double)cen[3 * (size_t)p + best_axis] - clo) * scale);
                b = std::min(std::max(b, 0), kBins - 1);
                return b < best_split;
            });
            mid = (uint32_t)(it - (idx.begin() + first));
        }
        if (best_axis < 0 || mid == 0 || mid == n) {
            // object median on the widest centroid axis (ties by triangle id)
            int axis = 0;
            for (int a = 1; a < 3; ++a)
                if ((double)cb.hi[a] - cb.lo[a] > (double)cb.hi[axis] - cb.lo[axis]) axis = a;
            mid = n / 2;
            std::nth_element(idx.begin() + first, idx.begin() + first + mid, idx.begin() + first + n,
                             [&](uint32_t x, uint32_t y) {
                                 float cx = cen[3 * (size_t)x + axis], cy = cen[3 * (size_t)y + axis];
                                 return cx < cy || (cx == cy && x < y);
                             });
        }
        uint32_t L = alloc(), R = alloc();
        nd.left = (int32_t)L;
        nd.right = (int32_t)R;
        bool par = n >= kParallelMin && threads_left.fetch_sub(1) > 0;
        if (par) {
            auto fut = std::async(std::launch::async, [this, L, first, mid, depth] { build(L, first, mid, depth + 1); });
            build(R, first + mid, n - mid, depth + 1);
            fut.get();
            threads_left.fetch_add(1);
        } else {
            if (n >= kParallelMin) threads_left.fetch_add(1);
            build(L, first, mid, depth + 1);
            build(R, first + mid, n - mid, depth + 1);
        }
    }
};

int32_t leaf_code(const BNode& b) {
    return (int32_t)~((b.first << 3) | (b.count - 1));
}

}  // namespace

bool build_bvh(const float* tris, uint32_t ntri, HostBvh& out, std::string& err) {
    out = HostBvh();
    if (ntri > kMaxTris) {
        err = "too many triangles";
        return false;
    }
    BvhNode empty_root;
    for (int i = 0; i < 12; ++i) empty_root.f[i] = (i % 2 == 0) ? INFINITY : -INFINITY;
    empty_root.c[0] = empty_root.c[1] = kEmpty;
    empty_root.c[2] = empty_root.c[3] = 0;
    if (ntri == 0) {
        out.nodes.push_back(empty_root);
        collapse_bvh4(out.nodes, out.nodes4, out.max_depth4);
        out.quant_ok = quantize_bvh4(out.nodes4, out.nodes4q);
        return true;
    }
    Builder b;
    b.tris = tris;
    try {
        b.tlo.resize(3 * (size_t)ntri);
        b.thi.resize(3 * (size_t)ntri);
        b.cen.resize(3 * (size_t)ntri);
        b.idx.resize(ntri);
        b.nodes.resize(2 * (size_t)ntri + 1);
    } catch (...) {
        err = "host allocation failed";
        return false;
    }
    for (uint32_t i = 0; i < ntri; ++i) {
        const float* v = tris + 9 * (size_t)i;
        for (int a = 0; a < 3; ++a) {
            float x0 = v[a], x1 = v[3 + a], x2 = v[6 + a];
            b.tlo[3 * (size_t)i + a] = std::min(x0, std::min(x1, x2));
            b.thi[3 * (size_t)i + a] = std::max(x0, std::max(x1, x2));
            b.cen[3 * (size_t)i + a] = (float)(((double)x0 + (double)x1 + (double)x2) / 3.0);
        }
        b.idx[i] = i;
    }
    b.threads_left = (int)std::max(1u, std::min(32u, std::thread::hardware_concurrency())) - 1;
    uint32_t root = b.alloc();
    b.build(root, 0, ntri, 0);

    // number inner nodes depth-first (left subtree right after its parent)
    const BNode& rn = b.nodes[root];
    double root_area = rn.box.half_area();
    if (!(root_area > 0.0)) root_area = 1.0;
    if (rn.left < 0) {
        BvhNode n = empty_root;
        const Box& bx = rn.box;
        n.f[0] = bx.lo[0]; n.f[1] = bx.hi[0]; n.f[2] = bx.lo[1]; n.f[3] = bx.hi[1];
        n.f[8] = bx.lo[2]; n.f[9] = bx.hi[2];
        n.c[0] = leaf_code(rn);
        out.nodes.push_back(n);
        out.max_leaf = rn.count;
        out.sah_cost = rn.count;
    } else {
        std::vector<uint32_t> stack{root};
        std::vector<int32_t> index(b.nnodes.load(), -1);
        // pass 1: preorder numbering of inner nodes
        std::vector<uint32_t> pre;
        while (!stack.empty()) {
            uint32_t x = stack.back();
            stack.pop_back();
            const BNode& nd = b.nodes[x];
            if (nd.left < 0) continue;
            index[x] = (int32_t)pre.size();
            pre.push_back(x);
            stack.push_back((uint32_t)nd.right);
            stack.push_back((uint32_t)nd.left);
        }
        out.nodes.resize(pre.size());
        double cost = 0.0;
        for (size_t k = 0; k < pre.size(); ++k) {
            const BNode& nd = b.nodes[pre[k]];
            const BNode& A = b.nodes[nd.left];
            const BNode& B = b.nodes[nd.right];
            BvhNode& o = out.nodes[k];
            o.f[0] = A.box.lo[0]; o.f[1] = A.box.hi[0]; o.f[2] = A.box.lo[1]; o.f[3] = A.box.hi[1];
            o.f[4] = B.box.lo[0]; o.f[5] = B.box.hi[0]; o.f[6] = B.box.lo[1]; o.f[7] = B.box.hi[1];
            o.f[8] = A.box.lo[2]; o.f[9] = A.box.hi[2]; o.f[10] = B.box.lo[2]; o.f[11] = B.box.hi[2];
            o.c[0] = A.left < 0 ? leaf_code(A) : index[nd.left];
            o.c[1] = B.left < 0 ? leaf_code(B) : index[nd.right];
            o.c[2] = o.c[3] = 0;
            cost += nd.box.half_area() / root_area;
            for (const BNode* ch : {&A, &B})
                if (ch->left < 0) {
                    cost += ch->box.half_area() / root_area * ch->count;
                    out.max_leaf = std::max(out.max_leaf, ch->count);
                    out.max_depth = std::max(out.max_depth, ch->depth);
                }
        }
        out.sah_cost = cost;
    }
    out.order = std::move(b.idx);
    try {
        collapse_bvh4(out.nodes, out.nodes4, out.max_depth4);
        out.quant_ok = quantize_bvh4(out.nodes4, out.nodes4q);
    } catch (...) {
        err = "host allocation failed";
        return false;
    }
    return true;
}

}  // namespace pt

namespace pt {

void collapse_bvh4(const std::vector<BvhNode>& n2, std::vector<Bvh4Node>& n4, uint32_t& max_depth4) {
    // Which binary nodes become four-wide nodes: each inner binary node either roots a
    // four-wide node (cost: its surface area, the probability that a ray visits it) or is
    // opened, its two subtrees taking its place among the entries of the four-wide node above
    // it (at most four entries per node).  Leaves are entries wherever they land, so their
    // cost is fixed; the total area of the four-wide nodes is minimized by dynamic programming
    // over (binary node, entries available), children before parents (every child follows its
    // parent in the depth-first order of the binary nodes).
    struct Entry {
        float lo[3], hi[3];
        int32_t code;
    };
    auto half_area = [](const Entry& e) {
        const double dx = (double)e.hi[0] - e.lo[0], dy = (double)e.hi[1] - e.lo[1], dz = (double)e.hi[2] - e.lo[2];
        return dx * dy + dy * dz + dz * dx;
    };
    auto children = [&](int32_t k, Entry out[2]) {
        const BvhNode& b = n2[(size_t)k];
        out[0] = Entry{{b.f[0], b.f[2], b.f[8]}, {b.f[1], b.f[3], b.f[9]}, b.c[0]};
        out[1] = Entry{{b.f[4], b.f[6], b.f[10]}, {b.f[5], b.f[7], b.f[11]}, b.c[1]};
    };
    n4.clear();
    max_depth4 = 0;
    if (n2.empty()) return;
    const size_t nn = n2.size();
    // own[k]: area of binary node k's box (the union of its children's boxes)
    // cost[k][m-1]: least cost of covering subtree k with at most m entries (m = 1..4);
    // m = 1: k roots a four-wide node.  split[k][m-1]: entries given to child 0 when k is
    // opened (0: not opened; 255: k has one child, which takes all m)
    std::vector<double> cost(nn * 4);
    std::vector<uint8_t> split(nn * 4);
    std::vector<double> own(nn);
    auto entry_cost = [&](const Entry& e, int m) -> double {   // an entry with at most m slots
        if (e.code == kEmpty || e.code < 0) return 0.0;          // leaves cost the same anywhere
        return cost[(size_t)e.code * 4 + (size_t)(m - 1)];
    };
    for (size_t kk = nn; kk-- > 0;) {
        const int32_t k = (int32_t)kk;
        Entry two[2];
        children(k, two);
        const bool has0 = two[0].code != kEmpty, has1 = two[1].code != kEmpty;
        Entry u = two[0];
        for (int a = 0; a < 3; ++a) {
            u.lo[a] = std::min(two[0].lo[a], two[1].lo[a]);
            u.hi[a] = std::max(two[0].hi[a], two[1].hi[a]);
        }
        own[kk] = has0 && has1 ? half_area(u) : half_area(has0 ? two[0] : two[1]);
        // opened with m slots: the best division of the slots between the two children
        auto opened = [&](int m, int& best0) -> double {
            double best = std::numeric_limits<double>::infinity();
            best0 = 0;
            if (has0 && has1) {
                for (int m0 = 1; m0 < m; ++m0) {
                    const double c = entry_cost(two[0], m0) + entry_cost(two[1], m - m0);
                    if (c < best) {
                        best = c;
                        best0 = m0;
                    }
                }
            } else {
                best = entry_cost(has0 ? two[0] : two[1], m);
                best0 = has0 ? m : 0;
            }
            return best;
        };
        int b0 = 0;
        const double root = own[kk] + opened(4, b0);   // k roots a four-wide node over 4 slots
        cost[kk * 4 + 0] = root;
        split[kk * 4 + 0] = 0;
        for (int m = 2; m <= 4; ++m) {
            const double op = opened(m, b0);
            const bool open = op < root;   // opening k pays when its subtrees fill the slots more cheaply
            cost[kk * 4 + (size_t)(m - 1)] = open ? op : root;
            split[kk * 4 + (size_t)(m - 1)] = (uint8_t)(open ? (has0 && has1 ? b0 : 255) : 0);
        }
    }
    // the entries of binary node k placed with at most m slots (k opened or not)
    std::function<void(const Entry&, int, Entry*, int&)> place = [&](const Entry& e, int m, Entry* out, int& ne) {
        if (e.code == kEmpty) return;
        if (e.code < 0 || m == 1) {
            out[ne++] = e;
            return;
        }
        const uint8_t s = split[(size_t)e.code * 4 + (size_t)(m - 1)];
        if (s == 0) {
            out[ne++] = e;
            return;
        }
        Entry two[2];
        children(e.code, two);
        if (s == 255) {   // one child only: it takes all m slots
            place(two[0].code != kEmpty ? two[0] : two[1], m, out, ne);
            return;
        }
        place(two[0], s, out, ne);
        place(two[1], m - s, out, ne);
    };
    struct Item {
        int32_t k2;       // binary node that roots a four-wide node
        uint32_t slot;    // four-wide node it becomes
        uint32_t depth;
    };
    n4.emplace_back();
    std::vector<Item> stack{{0, 0, 1}};
    while (!stack.empty()) {
        const Item it = stack.back();
        stack.pop_back();
        max_depth4 = std::max(max_depth4, it.depth);
        Entry e[4];
        int ne = 0;
        Entry two[2];
        children(it.k2, two);
        const bool has0 = two[0].code != kEmpty, has1 = two[1].code != kEmpty;
        if (has0 && has1) {
            int b0 = 0;
            double best = std::numeric_limits<double>::infinity();
            for (int m0 = 1; m0 < 4; ++m0) {
                const double c = entry_cost(two[0], m0) + entry_cost(two[1], 4 - m0);
                if (c < best) {
                    best = c;
                    b0 = m0;
                }
            }
            place(two[0], b0, e, ne);
            place(two[1], 4 - b0, e, ne);
        } else if (has0 || has1) {
            place(has0 ? two[0] : two[1], 4, e, ne);
        }
        Bvh4Node nd;
        for (int j = 0; j < 4; ++j) {
            nd.pad[j] = 0;
            if (j < ne) {
                nd.lx[j] = e[j].lo[0]; nd.hx[j] = e[j].hi[0];
                nd.ly[j] = e[j].lo[1]; nd.hy[j] = e[j].hi[1];
                nd.lz[j] = e[j].lo[2]; nd.hz[j] = e[j].hi[2];
                nd.c[j] = e[j].code;
            } else {
                nd.lx[j] = nd.ly[j] = nd.lz[j] = INFINITY;
                nd.hx[j] = nd.hy[j] = nd.hz[j] = -INFINITY;
                nd.c[j] = kEmpty;
            }
        }
        // inner children get the next slots, visited child 0 first
        for (int j = 0; j < ne; ++j)
            if (e[j].code >= 0) {
                const uint32_t slot = (uint32_t)n4.size();
                n4.emplace_back();
                nd.c[j] = (int32_t)slot;
            }
        for (int j = ne - 1; j >= 0; --j)
            if (e[j].code >= 0) stack.push_back(Item{e[j].code, (uint32_t)nd.c[j], it.depth + 1});
        n4[it.slot] = nd;
    }
}


bool quantize_bvh4(const std::vector<Bvh4Node>& n4, std::vector<Bvh4QNode>& q) {
    bool ok = true;
    q.assign(n4.size(), Bvh4QNode{});
    for (size_t i = 0; i < n4.size(); ++i) {
        const Bvh4Node& n = n4[i];
        Bvh4QNode& o = q[i];
        const float* lo4[3] = {n.lx, n.ly, n.lz};
        const float* hi4[3] = {n.hx, n.hy, n.hz};
        float lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
        bool any = false;
        for (int j = 0; j < 4; ++j) {
            o.c[j] = n.c[j];
            if (n.c[j] == kEmpty) continue;
            any = true;
            for (int a = 0; a < 3; ++a) {
                lo[a] = std::min(lo[a], lo4[a][j]);
                hi[a] = std::max(hi[a], hi4[a][j]);
            }
        }
        uint32_t ql[3] = {0, 0, 0}, qh[3] = {0, 0, 0};
        int e[3] = {0, 0, 0};
        if (any) {
            for (int a = 0; a < 3; ++a) {
                // the smallest step 2^e that spans the node in at most 255 steps (upper bound of the extent)
                const double ext = std::nextafter((double)hi[a] - (double)lo[a], INFINITY);
                int ea = -100;
                if (ext > 0.0) {
                    // a flat extent makes ext a denormal whose 255th part is 0: log2 = -inf, which
                    // must not reach the int conversion (clamped in double first)
                    const double lg = std::ceil(std::log2(ext / 255.0));
                    if (lg > -100.0) ea = (int)lg;
                }
                while (std::ceil(ext / std::ldexp(1.0, ea)) > 255.0) ++ea;
                if (ea > kQMaxExp) {
                    ok = false;
                    ea = kQMaxExp;   // the node is unusable; keep the byte in range
                }
                e[a] = ea;
                const double step = std::ldexp(1.0, ea);
                for (int j = 0; j < 4; ++j) {
                    uint32_t l = 255, h = 0;
                    if (n.c[j] != kEmpty) {
                        // differences bounded outward (one ulp beyond a rounded double), so that
                        // p + l * step <= child lo and p + h * step >= child hi hold exactly
                        const double dl = std::max(0.0, std::nextafter((double)lo4[a][j] - (double)lo[a], -INFINITY));
                        const double dh = std::nextafter((double)hi4[a][j] - (double)lo[a], INFINITY);
                        l = (uint32_t)std::min(255.0, std::floor(dl / step));
                        h = (uint32_t)std::min(255.0, std::ceil(dh / step));
                    }
                    ql[a] |= l << (8 * j);
                    qh[a] |= h << (8 * j);
                }
            }
        } else {
            for (int a = 0; a < 3; ++a) {
                lo[a] = 0.0f;
                ql[a] = 0xFFFFFFFFu;
                qh[a] = 0u;
            }
        }
        o.px = lo[0];
        o.py = lo[1];
        o.pz = lo[2];
        o.sx = std::ldexp(1.0f, e[0]);
        o.sy = std::ldexp(1.0f, e[1]);
        o.sz = std::ldexp(1.0f, e[2]);
        o.qlx = ql[0];
        o.qhx = qh[0];
        o.qly = ql[1];
        o.qhy = qh[1];
        o.qlz = ql[2];
        o.qhz = qh[2];
    }
    return ok;
}

}  // namespace pt
