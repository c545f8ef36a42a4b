// Internal declarations of libpt (not part of the C ABI).
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/pt.h"

namespace pt {

// Child-pair BVH2 node, 64 bytes: the boxes of both children and their codes.
//   f[0..3]  = c0.lo.x c0.hi.x c0.lo.y c0.hi.y
//   f[4..7]  = c1.lo.x c1.hi.x c1.lo.y c1.hi.y
//   f[8..11] = c0.lo.z c0.hi.z c1.lo.z c1.hi.z
//   i[12]    = code of c0, i[13] = code of c1, i[14..15] = 0
// code >= 0: inner node index; code == kEmpty: no child;
// otherwise leaf: ~code = (first << 3) | (count - 1), triangles [first, first+count)
// of the BVH-ordered triangle array.
constexpr int32_t kEmpty = INT32_MIN;
constexpr int kMaxLeaf = 4;
constexpr int kMaxDepth = 64;   // the traversal stack holds at most kMaxDepth entries
constexpr uint32_t kMaxTris = (1u << 28) - 2;

struct BvhNode {
    float f[12];
    int32_t c[4];
};
static_assert(sizeof(BvhNode) == 64, "node size");

// Four-wide node, 128 bytes: the boxes of up to four children (structure of arrays) and
// their codes (same code convention; kEmpty for an unused slot).
struct Bvh4Node {
    float lx[4], hx[4], ly[4], hy[4], lz[4], hz[4];
    int32_t c[4];
    int32_t pad[4];
};
static_assert(sizeof(Bvh4Node) == 128, "node size");

constexpr int kQMaxExp = 60;

// Quantized four-wide node, 64 bytes: the child boxes of the four-wide node of the same
// index as 8-bit steps of 2^e (one e per axis) above the node's lower corner p, rounded
// outward so that, in exact arithmetic, p + q * 2^e encloses every child box (8-bit child
// boxes relative to the parent, after Ylitie, Karras and Laine, HPG 2017).
struct Bvh4QNode {
    float px, py, pz;          // grid origin: the lower corner of the node's box
    float sx;                  // step along x: 2^e_x, -100 <= e_x <= kQMaxExp
    int32_t c[4];              // child codes as in Bvh4Node
    uint32_t qlx, qhx, qly, qhy;   // byte j: child j's lower / upper plane in steps
    uint32_t qlz, qhz;             // an empty child has lower 255, upper 0
    float sy, sz;              // steps along y and z
};
static_assert(sizeof(Bvh4QNode) == 64, "node size");

struct HostBvh {
    std::vector<BvhNode> nodes;
    std::vector<Bvh4Node> nodes4;  // the same tree collapsed to four children per node
    std::vector<Bvh4QNode> nodes4q; // the four-wide nodes with quantized child boxes
    bool quant_ok = true;          // every quantization exponent is at most kQMaxExp
    std::vector<uint32_t> order;   // BVH slot -> original triangle id
    uint32_t max_depth = 0;
    uint32_t max_leaf = 0;
    double sah_cost = 0.0;
    uint32_t max_depth4 = 0;       // inner-node depth of the four-wide tree
};

// Collapses the child-pair tree into four-wide nodes: a node's children are expanded,
// largest surface area first, into their own children until there are four or only
// leaves are left.  Leaf codes (triangle ranges) are unchanged.
void collapse_bvh4(const std::vector<BvhNode>& n2, std::vector<Bvh4Node>& n4, uint32_t& max_depth4);

// Quantizes the child boxes of the four-wide nodes (same order, same codes); returns false
// when some node needs a step above 2^kQMaxExp (its nodes are then not to be used).
bool quantize_bvh4(const std::vector<Bvh4Node>& n4, std::vector<Bvh4QNode>& q);

// Binned-SAH build over the triangles (host, multi-threaded, deterministic output).
bool build_bvh(const float* tris, uint32_t ntri, HostBvh& out, std::string& err);

}  // namespace pt
