// Shared declarations of the leaf-tile kernels (plain FP32 and MFMA
// filter): output sinks and the MFMA filter's arguments.
#pragma once

#include "tree.h"

namespace fnn {

struct TileOut {
    int32_t *deg;                 // count pass
    unsigned long long *cursor;   // fill pass: next free slot of each row
    int32_t *col;
    float *dist;
    // [0] pairs evaluated exactly, [1] FP64 rechecks, [2] pairs screened by
    // the MFMA filter, [3] filter survivors, [4] edges the filter would have
    // dropped (validate; must stay 0), [5] max relative distance error
    // (float bits, validate)
    unsigned long long *cnt;
    unsigned long long nnz;       // fill pass: slots available
    int *err;                     // fill pass: a write would leave the CSR
    // learned schedule: per-row slot end (slots of row r end at row_end[r]);
    // a row that would pass it is flagged in ovf and not written
    const int64_t *row_end;
    int32_t *ovf;
    // restricted fill: only rows with row_filter[r] != 0 are written
    const int32_t *row_filter;
    // learned schedule: entries beyond a row's slots go to a spill list
    int2 *spill;                  // (row, col) input ids
    float *spill_dist;
    unsigned long long *spill_cnt;
    unsigned long long spill_cap;
    // edge-list count pass: every edge (input ids, distance) is appended in
    // both directions while it fits; the running count may exceed the
    // capacity
    int2 *elist;
    float *edist;
    unsigned long long *ecnt;
    unsigned long long ecap;
    // work order (learned schedule): item k of the pass is inter[order[k]],
    // and work-groups take items through the counter next (each takes the
    // next item as it becomes free); null: inter in order, grid stride
    const uint32_t *order;
    unsigned long long *next;
};

struct GramArgs {
    int nn, npacks, nunits, nlist, kq;
    const void *q;        // quantised rows [n][kq] (tree order)
    const float *hx;      // (1 - c1) |x - mu|^2 per point
    float e2f;            // eps^2 in key space, slightly enlarged
    float gscale;         // 1 / scale^2 (FP8 global scale)
    Thr E;
    // batch of clouds: per-cloud thresholds by the cloud of a tree position
    // (null for a single cloud: e2f and E above apply)
    const CloudThr *ct;
    const int32_t *pcl;
    int fp64_dist, validate;
    const int32_t *lg, *lb, *ubeg;  // work lists: group, B pack, unit starts
    const int32_t *q_pb, *q_pe, *perm;
    // survivor list: (i, j | passed << 31) tree positions
    int2 *surv;
    unsigned long long *nsurv;     // running count (may exceed cap)
    long long surv_cap;
    // exact integer filter (Hamming codes, not validating): the survivors
    // are the edges, and degp counts the edges of each tree position; null
    // otherwise
    int32_t *degp;
    // screened pairs when the work list is every pair of one cloud
    // (n (n - 1) / 2, known in closed form); -1 otherwise (counted on the
    // device)
    long long dense_pairs;
    // survivor decisions: where non-null, the ranks the degree counters
    // returned for an edge's two endpoints (slot i, like the edge), so the
    // fill places it without a cursor
    int2 *erank;
    // filter on leading principal coordinates: their number (0: off), the
    // factor applied to eps^2 (1 when off) and the captured variance
    int proj;
    double t2mul;
    double e2add;         // added to the filter's (scaled) eps^2 (FP16 subnormals)
    double captured;
    // bichromatic query: only pairs across the two clouds are evaluated
    int cross;
    // narrow 16-bit rows copied per pack (64 rows each, zero past the pack)
    // and their column terms 0.5 hx (FLT_MAX past the pack); null when the
    // staged kernel runs
    const void *qp;
    const float *ayp;
    // uniform packs over one cloud: pack k holds tree positions GP k ..
    // min(GP k + GP, upk) - 1 and a work unit's B packs are consecutive;
    // 0: packs from q_pb / q_pe and the list
    int upk;
};

// Per-pack copies of the quantised rows and column terms for the narrow
// 16-bit kernel (G.qp, G.ayp), when that kernel applies; needs G.q, G.hx,
// G.kq, G.q_pb, G.q_pe, G.nn, G.npacks.
void gram_pad_packs(int metric, int prec, GramArgs &G, Scratch &S);
// Exact decision of the survivor list: edges[i] and edist[i] (input ids,
// FP32 distance) for survivor i, (-1, -1) when it is no edge, and per-row
// degrees; counts land in out.cnt.
void survivors_launch(int metric, const Pts &P, const GramArgs &G,
                      long long nsurv, int2 *edges, float *edist, const TileOut &o,
                      hipStream_t s);
// Edge list (input ids, distance; (-1, -1) entries skipped) into the CSR:
// both: every edge listed once, written into both rows; else every edge
// listed in both directions, each entry written into its first id's row.
void edges_scatter(const int2 *edges, const float *edist, long long ne, bool both,
                   const TileOut &o, hipStream_t s);
// Decided survivors into the CSR without cursors: edge i goes to slots
// row_ptr[a] + ranks[i].x of row a and row_ptr[b] + ranks[i].y of row b, the
// ranks its degree counters returned (each in [0, degree), so the rows
// fill exactly); a rank past its row sets ERR_INDEX.
void edges_place(const int2 *edges, const float *edist, const int2 *erank, long long ne,
                 const int64_t *row_ptr, const TileOut &o, hipStream_t s);
// Survivors of the exact integer filter (tree positions) into the CSR, with
// their Hamming distances.
void edges_scatter_ham(const int2 *surv, long long ne, const Pts &P,
                       const int32_t *perm, const TileOut &o, hipStream_t s);
// deg[perm[p]] += degp[p] for every tree position p; *dsum += sum degp.
void degrees_from_positions(const int32_t *degp, const int32_t *perm, int n,
                            int32_t *deg, unsigned long long *dsum, hipStream_t s);

// 2 c1 mean|x - mu|^2 / t2min for the BF16 filter (mu per cloud): how much
// its rounding margin widens the test against the smallest squared
// threshold; small values mean a selective filter.
// Per-query statistics of the rows the filter quantises, computed once by
// the automatic precision rule and reused by the quantisation: the cloud
// centres (column sums and 1 / sizes) and the largest |x - mu|.
struct GramPre {
    const float *sums = nullptr;
    const float *inv = nullptr;
    float absmax = 0.f;
    bool have = false;
};
double gram_margin_ratio(const fnn_tree *T, double t2min, int prec, Scratch &S,
                         GramPre *pre = nullptr);

// True when no query pack exceeds the filter's tile height (the work list
// of every pack pair then exists in closed form).
bool gram_packs_fit(const fnn_tree *T, Scratch &S);

// Squared threshold of the filter's key (eps^2, or the squared chord of
// the angular threshold).
double gram_t2(int metric, double eps, const Thr &E);
// eps^2 in the filter's key space times t2mul, slightly enlarged so that the
// FP32 evaluation of the filter test itself cannot flip a true edge.
float gram_eps2(int metric, double eps, const Thr &E, double t2mul = 1.0, double add = 0.0);

// proj: leading principal coordinates for the filter (-1 off, 0 automatic,
// else their number); t2min: smallest squared threshold of the query.
void gram_prepare(const fnn_tree *T, int prec, int proj, double eps, const Thr &E,
                  double t2min, const int2 *inter, long long ninter, Scratch &S,
                  GramArgs &G, int2 **rest, long long *nrest,
                  const GramPre *pre = nullptr);
void gram_launch(int metric, int prec, bool fill_pass, const Pts &P,
                 const GramArgs &G, const TileOut &o, hipStream_t s);

}  // namespace fnn
