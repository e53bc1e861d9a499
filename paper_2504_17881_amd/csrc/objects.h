// Host objects behind the opaque ABI handles.
#pragma once

#include <stdint.h>

#include <vector>

#include "internal.h"

struct prx_ham {
    int n = 0;
    std::vector<uint64_t> x, z;
    std::vector<double> h;
};

struct prx_sched {
    int n = 0;
    std::vector<uint64_t> x, z;
    std::vector<double> phi;
};

namespace prx {

// A rotation as the kernels apply it (after splitting large angles).
struct KRot {
    uint64_t x, z;
    double phi;
    size_t src;  // index in the schedule
};

// Rotation record before conversion to the state's precision.
struct RotRecD {
    uint64_t z = 0, zhigh = 0;
    uint32_t info = 0;
    double tau_a = 0.0, tau_b = 0.0;
    bool fold = false;  // device tau_a is -tau_a (static-sign variant with zeta_slot set)
};

enum PassKind { kPlain = 0, kSpan = 1, kTile = 2, kPerm = 3 };

struct Pass {
    int kind = kPlain;
    size_t r0 = 0, r1 = 0;  // kernel rotations [r0, r1)
    // span
    int m = 0;
    uint64_t basis[kMaxChunkRank] = {};
    uint32_t pivot[kMaxChunkRank] = {};
    double fscale[kMaxChunkRank] = {1, 1, 1, 1, 1, 1};
    // tile
    int B = 0, b = 0, g = 0;
    uint64_t vmask[kMaxVirtual] = {};
    uint32_t tpivot[kMaxVirtual] = {};
    size_t c0 = 0, c1 = 0;  // chunks
    double scale = 1.0;
    bool norm_out = false, renorm_in = false;
    // relabelling (kPerm): index bit ppos[j] moves to index bit ppos[pdst[j]]
    uint32_t ppos[kPermBits] = {};
    uint8_t pdst[kPermBits] = {};
};

struct PlanCfg {
    int B = 12;           // tile qubits
    int m = 4;            // chunk rank (tile)
    int span_m = 4;       // max span rank
    int max_fuse = 64;
    int max_virtual = 2;
    int renorm_every = 1;
    bool commuting = false;
    bool span_only = false;  // batched plans: every pass is a span pass ...
    int pad_rank = 0;        // ... whose basis is padded to exactly this rank
    bool tile_only = false;  // batched plans: every pass is a tile pass
    bool relabel = false;    // qubit-relabelling passes between segments
    unsigned grid_cap = (unsigned)kMaxGridBlocks;  // workgroups per sweep launch
};

// Kernel arguments of a tile pass of a plan for n qubits.
void tile_args(int n, const Pass &ps, TileArgs &a);

// Workspace regions (byte offsets, 256-aligned).
struct WsLayout {
    size_t rot_off = 0, rot_bytes = 0;
    size_t chunk_off = 0, chunk_bytes = 0;
    size_t part_off = 0, part_bytes = 0;
    size_t scal_off = 0, scal_bytes = 0;
    size_t total = 0;
};

}  // namespace prx

struct prx_plan {
    int n = 0;
    prx_dtype dtype = PRX_C128;
    prx_kernel kernel = PRX_PLAIN;
    size_t begin = 0, end = 0;
    prx::PlanCfg cfg;
    std::vector<prx::KRot> rots;
    std::vector<prx::Pass> passes;
    std::vector<prx::ChunkRec> chunks;
    std::vector<unsigned char> rot_table;  // RotRec<float> or RotRec<double> image
    prx::WsLayout ws;
    size_t plain_passes = 0, span_passes = 0, tile_passes = 0;
};
