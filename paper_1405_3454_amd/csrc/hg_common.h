// Internal definitions shared by the library's own kernels and host code.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace hg {

constexpr int WAVE = 64;
constexpr int PTS_PER_LANE = 4;                 // one float4 of x and of y per lane
constexpr int CHUNK = WAVE * PTS_PER_LANE;      // 256 consecutive points per wave step
constexpr int TILE_CHUNKS = 4;
constexpr int TILE = CHUNK * TILE_CHUNKS;       // 1024 points: unit of the filter passes
constexpr int TILE_WORDS = TILE / 64;           // survivor mask words per tile
constexpr int FIXED_SLOTS = 16;
constexpr int MAX_DIRS = 8;                     // learned extra directions per set
constexpr int MAX_SLOTS = FIXED_SLOTS + MAX_DIRS;
constexpr int SPAN_ROWS = 256;                  // quick-accept rows per polygon
constexpr uint32_t NONE = 0xFFFFFFFFu;
constexpr float GRIDF = 16777216.0f;            // 2^24
constexpr double GRIDD = 16777216.0;

// Filter polygon of one set, in grid units (coordinate * 2^24, integers).
// Edge e is strictly satisfied by p iff
//     E_e(p) = fma(ex, py, fma(-ey, px, c)) > 0,   c = ey*ax - ex*ay,
// exact in binary64 on the grid (|E| < 2^51).  Unused edges hold (0, 0, 1);
// a polygon with fewer than 3 vertices has edge 0 = (0, 0, -1), so nothing
// is strictly inside it.
struct Poly {
    double ex[MAX_SLOTS];
    double ey[MAX_SLOTS];
    double c[MAX_SLOTS];
    uint32_t verts[MAX_SLOTS];
    int32_t m;
    int32_t ky_lo;      // quick-accept rows cover ky in [ky_lo, ky_lo + yspan]
    int32_t yspan;      // < 0: no quick-accept rows (and nothing strictly inside)
    int32_t shift;      // row = (ky - ky_lo) >> shift
    int32_t ymin, ymax; // the polygon's y-range (grid units)
    int32_t pad[2];
    int32_t vx[MAX_SLOTS], vy[MAX_SLOTS];   // vertices (grid units); edge e runs from e to e + 1
};

// One row of the polygon's y-range (ky in [y0, y1]), as two integer ranges
// tested with one unsigned comparison each, (uint32)(kx - start) <= width:
//  - quick-accept span [xl, xl + xw]: every grid point of the row in it is
//    strictly inside the polygon (verified exactly at the rectangle's
//    corners; no span: xl = SPAN_FAR);
//  - extent [ob, ob + ow]: the grid points strictly between the polygon's
//    x-extent over the row, widened by a grid unit on each side; a point of
//    the row outside it is not strictly inside the polygon.
// Per row a second word lists the edges whose y-range meets the row (one byte
// each, ROW_EDGE_NONE = unused, ROW_EDGES_ALL = more than four): for a point
// of the row, being strictly inside those edges is the same as being
// strictly inside the polygon.
struct Span {
    int32_t xl, xw, ob, ow;
};
constexpr int32_t SPAN_FAR = 1 << 30;           // start of an empty range (kx < 2^24)
constexpr uint32_t ROW_EDGE_NONE = 31;          // index of an always-satisfied edge
constexpr uint32_t ROW_EDGES_ALL = 0xFFFFFFFFu;

// QuickHull refinement of the survivors (hull stage): rounds, edge slots per
// set and round, and the per-survivor edge states besides an edge id.
constexpr int REF_ROUNDS = 4;
constexpr int RE_CAP = MAX_SLOTS << REF_ROUNDS;
constexpr uint16_t RE_NONE = 0xFFFF;              // kept, not assigned to an edge
constexpr uint16_t RE_DROP = 0xFFFE;              // strictly inside the hull

// A refinement edge a->b in grid units; ax == INT32_MIN: empty slot.
struct REdge {
    int32_t ax, ay, bx, by;
};
__host__ __device__ inline REdge redge_empty() { return REdge{INT32_MIN, 0, 0, 0}; }


// Kernel kinds for the per-kernel event timer.
enum Kind {
    K_TILEMAP = 0, K_EXTREMES, K_POLYGON, K_DISCARD, K_SCAN, K_SCATTER,
    K_KEYS, K_SORT_HIST, K_SORT_SCAN, K_SORT_SCATTER, K_CHAIN, K_CHAIN_COMPACT,
    K_FINAL, K_LOOKUP, K_VALIDATE, K_MISC, K_HIST32, K_MLP, K_LABELS, K_REFINE, K_REFINE_SPLIT, K_NKINDS
};

// Direction presets (rotation groups of Step 1).  Preset 0: 0/30/45/60
// degrees; preset 1: 0/30/75/120 (its last group repeats the 30-degree one);
// preset 1 + G (G = 1..6): G groups at 90 j / G degrees, 4G evenly spaced
// extreme directions (G = 1: the min/max x and y quadrilateral).
constexpr int NUM_PRESETS = 8;
constexpr int MAX_GROUPS = 6;
__host__ __device__ constexpr int preset_groups(int P) { return P <= 1 ? 4 : P - 1; }
// groups the extremes pass evaluates (preset 1 copies its fourth group)
__host__ __device__ constexpr int preset_eval_groups(int P) { return P == 1 ? 3 : preset_groups(P); }
// fixed slot positions: at least 16, so that learned slots start at 16 when
// the fixed table has no more than 16 slots; unused positions hold NONE
__host__ __device__ constexpr int preset_fixed_slots(int P) {
    return 4 * preset_groups(P) > FIXED_SLOTS ? 4 * preset_groups(P) : FIXED_SLOTS;
}

// Direction constants for one launch.  Preset groups: (gc[g], gs[g]).
struct Dirs {
    double gc[MAX_GROUPS];
    double gs[MAX_GROUPS];
};

}  // namespace hg
