// Internal interface between the host runtime (sj_runtime.cpp) and the HIP
// kernels (sj_kernels.hip, sj_join.hip). Not part of the public C ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace sj {

constexpr int kMaxJCols = 8;    // distinct join columns of one relation
constexpr int kMaxProbe = 8;    // filters probed by one scan
constexpr int kMaxBuild = 8;    // filters built by one scan
constexpr int kMaxK = 12;       // bits per key

constexpr int kSieveBlock = 256;
constexpr int kSieveItems = 8;
constexpr int kSieveTile = kSieveBlock * kSieveItems;

// Sieve scans (probe and compaction) run one 1024-thread workgroup per CU, so a
// workgroup can hold a filter of up to kLdsFilterBytes in LDS; workgroup b owns a
// contiguous run of tiles. With the probe's static LDS (a 32 KB answer cache and 16 KB
// of live-row lists) that stays within the 160 KB of a CU.
constexpr int kProbeBlock = 1024;
constexpr uint32_t kProbeGrid = 256;       // default workgroups of a probe / compaction launch
constexpr uint32_t kProbeGridMax = 1024;
constexpr int kProbeTile = kProbeBlock * kSieveItems;
constexpr uint32_t kLdsFilterBytes = 108 * 1024;

constexpr int kScanBlock = 256;
constexpr int kScanItems = 8;
constexpr int kScanTile = kScanBlock * kScanItems;

constexpr int kRadixBits = 8;
constexpr int kRadixBins = 1 << kRadixBits;
constexpr int kRadixPasses = 64 / kRadixBits;   // a 64-bit composite key at most
constexpr int kRadixBlock = 256;
constexpr int kRadixItems = 8;
constexpr int kRadixTile = kRadixBlock * kRadixItems;
// Lists of up to kRadixSmallN entries are sorted in tiles of kRadixItemsSmall items per
// thread: more workgroups take part (a 390K-entry list is 762 tiles instead of 191),
// while larger lists keep the larger tiles and their smaller per-tile histograms.
constexpr int kRadixItemsSmall = 2;
constexpr uint32_t kRadixSmallN = 1u << 20;
__host__ __device__ inline uint32_t radix_tile(uint32_t n) {
    return n <= kRadixSmallN ? static_cast<uint32_t>(kRadixBlock * kRadixItemsSmall) : static_cast<uint32_t>(kRadixTile);
}
// The most tiles a list of any n <= cap entries takes.
__host__ __device__ inline uint32_t radix_tiles_max(uint32_t cap) {
    const uint32_t small = cap < kRadixSmallN ? cap : kRadixSmallN;
    const uint32_t ts = kRadixBlock * kRadixItemsSmall;
    const uint32_t a = (small + ts - 1) / ts;
    const uint32_t b = (cap + kRadixTile - 1) / kRadixTile;
    return a > b ? a : b;
}

constexpr int kPersistentBlocks = 256 * 8;  // 256 CUs, a few resident blocks each

// Decoupled look-back state for one launch: one 64-bit status word per tile
// ((flag << 32) | count, flag 1 = the tile's own count, 2 = inclusive prefix) and a
// counter that hands out tile ids in order. Both must be zero before the launch.
struct Lookback {
    uint64_t *status;
    uint32_t *counter;
};

struct FilterRef {
    uint32_t *words;
    const uint32_t *nblocks;   // device-side block count
};

// One scan over a relation's rows (full columns) or over its current survivor list.
struct StepArgs {
    const uint32_t *src_rid;   // list source: row ids; nullptr: full scan, rid = row index
    const uint32_t *src_count; // list source: device-side row count
    uint32_t src_rows;         // full scan: number of rows
    int ncol;
    const int32_t *col[kMaxJCols];
    const int32_t *pred;       // full scan predicate column or nullptr
    int32_t pred_lo, pred_hi;
    int nprobe;
    int8_t probe_col[kMaxProbe];
    FilterRef probe[kMaxProbe];
    uint32_t *out_rid;         // nullptr: no survivor list is written
    int32_t *out_col[kMaxJCols];
    uint32_t *out_count;       // device-side survivor count (written when out_rid != nullptr)
    uint8_t *bits;             // [ceil(rows / 8)] survivor flags of the scan, 8 rows per byte
    uint32_t *counts;          // [grid] survivors per workgroup (two-launch form)
    Lookback lb;               // one-launch form: [grid] status words and the ticket counter, zeroed before
    uint32_t grid;             // workgroups of the probe and compaction launches
    uint32_t lds_words;        // LDS words set aside for one probed filter (0: none)
    uint32_t seed;
    int k;
    int logB;
};

// ---- launch wrappers (sj_kernels.hip) ----
hipError_t launch_zero(void *p, uint64_t bytes, hipStream_t s);

// Inserts into a built filter (Section 2.4): probe a batch of keys against the
// filter as it is (contained[i], and the count of keys it does not contain added to
// *missing); with `set`, the keys found missing then set their bits in place.
struct FilterUpdate {
    uint32_t *words;
    const uint32_t *nblocks;   // device-side block count (unchanged by inserts)
    const int32_t *keys;
    uint64_t n;
    uint8_t *contained;
    unsigned long long *missing;
    uint32_t seed;
    int k;
    int logB;
};
hipError_t launch_filter_update(const FilterUpdate &u, bool set, hipStream_t s);

// Counting twins of blocked filters (sj_update.hip): one 4-bit counter per bit position,
// block b's position p in nibble p % 8 of word b * B / 8 + p / 8; saturating at 15.
struct CfArgs {
    uint32_t *counts;
    uint32_t nblocks;
    const int32_t *keys;
    uint64_t n;
    const int32_t *pred;       // rows with pred < lo or >= hi are skipped (nullptr: none)
    int32_t pred_lo, pred_hi;
    uint32_t seed;
    int k;
    int logB;
};
// sign +1 inserts, -1 deletes; with n_dev the key count is read on the device (n_max bounds it)
hipError_t launch_cf_update(const CfArgs &a, const uint32_t *n_dev, uint32_t n_max, int sign, hipStream_t s);
hipError_t launch_cf_probe(const CfArgs &a, uint8_t *contained, unsigned long long *missing, hipStream_t s);
hipError_t launch_cf_export(const uint32_t *counts, uint64_t nwords, uint32_t *words, hipStream_t s);

// Propagation of inserted tuples toward the root (Section 2.4).
struct KeySet {
    uint64_t *slots;           // [mask + 1], zeroed before inserts; nullptr: no set (all rows qualify)
    uint32_t mask;
};
struct PropArgs {
    uint64_t nrows;
    const int32_t *match_col;  // key that must be in `set` (nullptr: none)
    KeySet set;
    const int32_t *pred;
    int32_t pred_lo, pred_hi;
    int nprobe;
    const int32_t *probe_col[kMaxProbe];
    FilterRef probe[kMaxProbe];
    const int32_t *out_col;    // key appended for each qualifying row
    int32_t *out;
    uint32_t *out_n;           // zeroed before
    uint32_t seed;
    int k;
    int logB;
};
hipError_t launch_propagate_rows(const PropArgs &a, hipStream_t s);
// Insert keys[i] for every i with !skip[i] (skip may be null) into the set.
hipError_t launch_set_insert(const KeySet &set, const int32_t *keys, const uint8_t *skip, uint64_t n,
                             hipStream_t s);
hipError_t launch_count_pred(const int32_t *col, uint32_t n, int32_t lo, int32_t hi, uint32_t *out,
                             hipStream_t s);
// A sieve step is two launches: the probe scan (survivor bits and per-workgroup counts)
// and, when the step writes a survivor list, the compaction.
hipError_t launch_sieve_probe(const StepArgs &a, uint32_t max_rows, hipStream_t s);
hipError_t launch_sieve_compact(const StepArgs &a, uint32_t max_rows, hipStream_t s);
// probe and survivor list in one launch (a.out_rid and a.lb required)
hipError_t launch_sieve_fused(const StepArgs &a, uint32_t max_rows, hipStream_t s);

// Partitioned build of one filter from a key column (full column with an optional
// predicate, or a survivor-list column with a device-side length).
constexpr int kBuildBlock = 1024;
// A build tile holds tile_of(n) keys: at least kBuildTileMin, and few enough that at
// most kBuildMaxTiles tiles cover the input. Few large tiles keep the scatter's runs
// per (region, tile) long (each such run costs about one partly written cache line)
// and let the tile's dedup cache drop more repeats.
constexpr uint32_t kBuildTileMin = kBuildBlock * 8;
constexpr uint32_t kBuildMaxTiles = 512;
__host__ __device__ inline uint32_t build_tile_of(uint32_t n) {
    const uint32_t per = (n + kBuildMaxTiles - 1) / kBuildMaxTiles;
    const uint32_t t = (per + kBuildTileMin - 1) / kBuildTileMin * kBuildTileMin;
    return t > kBuildTileMin ? t : kBuildTileMin;
}
constexpr uint32_t kRegionBytes = 16 * 1024;   // LDS per region workgroup (the largest region)
constexpr int kRegionThreads = 512;
// A filter is cut into at least kRegionsTarget regions when regions of kRegionMinShift
// (log2 blocks) or more allow it, so small filters still spread over the chip; the
// region count is then below max(blocks / largest region, 2 * kRegionsTarget).
constexpr uint32_t kRegionsTarget = 256;
constexpr uint32_t kRegionMinShift = 3;
__host__ __device__ constexpr uint32_t region_count_cap(uint64_t nblocks_max, uint32_t region_blocks) {
    const uint64_t big = (nblocks_max + region_blocks - 1) / region_blocks;
    return static_cast<uint32_t>(big > 2 * kRegionsTarget ? big : 2 * kRegionsTarget);
}
struct BuildArgs {
    const int32_t *keys;
    const uint32_t *n_dev;     // list source: device-side length; nullptr: use n
    uint32_t n;
    uint32_t n_max;            // capacity of the source
    const int32_t *pred;       // full-column source: predicate column or nullptr
    int32_t pred_lo, pred_hi;
    const uint32_t *nkeys_dev; // keys inserted (sizes the filter); nullptr: the source length
    uint32_t bits_per_key;
    uint32_t *words;
    uint32_t *nblocks;         // device-side filter size in blocks (written by the build)
    uint32_t nblocks_max;
    uint32_t region_blocks;    // kRegionBytes / (block bytes): the largest region (a power of two)
    uint32_t *hist;            // [regions * tiles] counts, then their exclusive prefix
    uint64_t *keep;            // [(n_max + tile) / 64] bit e: element e is staged
    uint32_t *stage;           // [n_max] staged keys, grouped by region
    uint32_t *total_dev;       // number of staged keys (zeroed before)
    Lookback lb;               // scan state (zeroed before)
    uint32_t seed;
    int k;
    int logB;
};
// The build's four launches, in order: 0 region counts per tile, 1 their scan, 2 the
// scatter into region buckets, 3 the per-region bit setting.
constexpr int kBuildStages = 4;
hipError_t launch_filter_build_stage(const BuildArgs &a, int stage, hipStream_t s);

// ---- join phase (sj_join.hip) ----
// A relation's sieved rows regrouped by its parent-edge key ("bucket order").
struct Buckets {
    uint32_t cap;              // capacity (rows)
    const uint32_t *n;         // device-side number of entries
    uint32_t *rid;             // [cap] row ids in bucket order
    int32_t *col[kMaxJCols];   // [cap] join-column values in bucket order
    int npay;
    int key_jcol;              // which join column is the bucket key
    uint32_t *dir_begin;       // [cap + 1] first entry of each distinct key, then n
    int32_t *dir_key;          // [cap]
    uint32_t *ndir;            // device-side number of distinct keys
    uint64_t *slots;           // hash index over dir keys, [slot_cap]
    uint32_t slot_cap;         // power of two
    uint32_t *slot_mask;       // device-side mask used (<= slot_cap - 1)
    uint64_t *cw;              // [cap + 1] exclusive prefix of entry weights (result counts)
    uint64_t *cv;              // [cap + 1] exclusive prefix of entry checksum weights
};

// LSD radix sort of (key, list index) pairs; the key is one 32-bit column, or two
// (primary, secondary) compared as the 64-bit (primary << 32) | secondary.
struct SortScratch {
    uint32_t cap;
    uint32_t *klo[2];          // ping-pong: low key word (the only word of 1-word keys)
    uint32_t *khi[2];          //            high key word (2-word keys)
    uint32_t *vals[2];
    uint32_t *hist;            // [kRadixBins * ntiles_max]
    uint32_t *ghist;           // [kRadixPasses * kRadixBins], zeroed
    uint32_t *ctl;             // [32] pass control words (written on device)
    Lookback lb[kRadixPasses]; // scan of each pass's histogram
};

// Sort the list (rid, cols) by column key_col (then by column sec_col when
// sec_col >= 0) into bucket order and build the directory (on key_col) and its hash
// index. list_count is the device-side list length.
hipError_t launch_build_buckets(const uint32_t *list_rid, const int32_t *const *list_cols, int ncol,
                                const uint32_t *list_count, int key_col, int sec_col, const Buckets &b,
                                const SortScratch &ss, Lookback lb_dir, hipStream_t s);

// Per-entry DP weights of a bucketed relation (or the root list), scanned into
// cw/cv. child[c] is the bucketed child joined on list column child_col[c].
// A thread holds ITEMS entries (tiles of kScanBlock * ITEMS entries) and looks them up
// in up to CH = kDpSlots / ITEMS children at once. Few entries per thread spread a
// relation of a few hundred thousand entries over many more workgroups than CUs: a
// relation with one child takes 2 entries per thread, one with more children 1 entry
// with all of its children looked up together.
constexpr int kDpSlots = 8;
inline int dp_items(int nchild) { return nchild <= 1 ? 2 : 1; }
inline uint32_t dp_tile(int nchild) { return static_cast<uint32_t>(kScanBlock * dp_items(nchild)); }

struct DpArgs {
    uint32_t rel;              // relation index (checksum factor)
    const uint32_t *n;         // device-side entries
    uint32_t cap;
    const uint32_t *rid;
    const int32_t *col[kMaxJCols];
    int nchild;
    int child_col[kMaxJCols];
    Buckets child[kMaxJCols];
    uint64_t *cw;              // [cap + 1]
    uint64_t *cv;              // [cap + 1]
    uint32_t *blo[kMaxJCols];  // [cap] per child: first entry of the matching child bucket
    uint32_t *bhi[kMaxJCols];  // [cap] per child: one past its last entry (lo = hi: none)
    uint32_t skip_mask;        // children whose totals are not multiplied in (bounds still kept)
    uint64_t *tile_sums;       // [2 * grid] per-run sums (grid <= ceil(cap / dp_tile(nchild)))
    uint64_t *totals;          // [2] result count and checksum, or nullptr
};
hipError_t launch_dp(const DpArgs &a, hipStream_t s);

// Materialisation over the join tree. Position x is the x-th relation in preorder
// (position 0 is the root); its entries are the root's survivor list or a bucketed
// relation's entries in bucket order.
constexpr int kMatMaxRels = 16;
// What the materialisation writes per tuple: row ids (n = 0: one per relation, in
// relation-index order) or projected values (n columns: output column q is column
// col[q] of relation rel[q] at the tuple's row of that relation).
constexpr int kMaxProj = 32;
struct Projection {
    int n;
    int rel[kMaxProj];
    const int32_t *col[kMaxProj];
};
struct MatArgs {
    int nrels;
    int order[kMatMaxRels];        // relation index at each position
    int parent_pos[kMatMaxRels];
    int is_leaf[kMatMaxRels];
    int nchild[kMatMaxRels];
    const uint32_t *rid[kMatMaxRels];   // row id of each entry
    const uint64_t *cw[kMatMaxRels];    // exclusive prefix of entry weights ([n + 1])
    const uint32_t *blo[kMatMaxRels];   // bucket of position x inside the parent's entry e:
    const uint32_t *bhi[kMatMaxRels];   //   [blo[x][e], bhi[x][e])
    const uint32_t *root_n;
    uint64_t count;                // total result tuples (host copy), used when count_dev is null
    const uint64_t *count_dev;     // device-side total, or nullptr
    uint64_t capacity;             // tuples `out` holds: nothing is written if the total exceeds it
    int32_t *out;
    Projection proj;               // row ids (proj.n = 0) or projected values
    // Factorised materialisation (launch_mat_table / launch_mat_output): position x's
    // table of the tuples below each of its entries, for non-root positions with
    // children (nullptr elsewhere): entry e's rows start at row cw[x][e], a row holds
    // the row ids of x's subtree in preorder (subtree[x] words).
    uint32_t *tab[kMatMaxRels];
    uint64_t tab_words[kMatMaxRels];   // words tab[x] can hold
    int subtree[kMatMaxRels];          // positions x .. x + subtree[x] - 1 form x's subtree
    const uint32_t *n_ent[kMatMaxRels];   // device-side entry count of each position
    int fact;                      // the factorised launches ran: launch_materialize then
                                   // writes only if some table did not fit its scratch
};
// Grid: enough blocks for min(count, capacity) tuples when the count is on the host;
// a fixed persistent grid over the output when it is read on the device.
hipError_t launch_materialize(const MatArgs &a, hipStream_t s);
// Factorised materialisation: the tables, deepest positions first (launch_mat_table for
// each non-root position with children, in decreasing position order), then the output
// as one expansion of the root (launch_mat_output). Usable when every position has at
// most kFactMaxChild children and each table position has its scratch (mat_factorisable);
// if some table does not fit its scratch, these launches write nothing and a following
// launch_materialize (with fact = 1) writes the output instead.
constexpr int kFactMaxChild = 4;
bool mat_factorisable(const MatArgs &a);
hipError_t launch_mat_table(const MatArgs &a, int x, hipStream_t s);
hipError_t launch_mat_output(const MatArgs &a, hipStream_t s);

// Cyclic joins whose closing edges all end at the last relation L of the preorder
// (a leaf): the other relations form a tree (the "prefix") whose tuples are
// enumerated; L is bucketed by (tree key, closing key), so a prefix's matches are the
// run of its L bucket whose closing column equals the prefix's closing value(s).
constexpr int kMaxClose = 4;
struct CycArgs {
    MatArgs m;                 // the prefix positions 0 .. n-2 (m.nrels = n - 1)
    int nrels;                 // output width n
    int L_rel;                 // relation index of L
    int pos_P;                 // position of L's parent
    const uint32_t *Lblo, *Lbhi;   // L's bucket below each entry of its parent
    const uint32_t *Lrid;
    const int32_t *Lclose;     // L's closing column in bucket order (ascending as u32 inside a bucket)
    const uint64_t *Lcv;       // exclusive prefix of L's checksum factors
    // closing edges ending at L on the column L is sorted by: their values on the prefix
    // must agree, and select the run of L's bucket that holds that value
    int nclose;
    int cpos[kMaxClose];       // position of each closing edge's other end
    const int32_t *ccol[kMaxClose];  // its closing column, entry-indexed
    // closing edges ending at L on another column: checked on each entry of the run
    int nextra;
    int xpos[kMaxClose];
    const int32_t *xcol[kMaxClose];  // the prefix side, entry-indexed
    const int32_t *xL[kMaxClose];    // L's column, in L's bucket order
    // closing edges between two prefix relations: checked on the prefix
    int ninner;
    int ipos[kMaxClose][2];
    const int32_t *icol[kMaxClose][2];
    uint64_t wpre;             // number of prefixes
    uint32_t G;                // threads; thread t takes an even share of the prefixes
    uint64_t *cnt;             // [G] results per thread
    uint64_t *chk;             // [G] checksum per thread
    uint64_t *off;             // [G] exclusive prefix of cnt (write pass)
    uint64_t *totals;          // [2] count, checksum
    int32_t *out;
};
hipError_t launch_cyclic_count(const CycArgs &a, hipStream_t s);
hipError_t launch_cyclic_write(const CycArgs &a, hipStream_t s);


// Directed 3-cycles root - P - L - root (tree edges root-P and P-L, closing edge
// L-root) counted by intersection instead of the binary plan's wedge expansion.
// A pair hash maps a relation's (key, key) pair to its row count and the sum of its
// rows' checksum factors. One slot past the table (index `cap`) holds the pair whose
// 64-bit key equals the empty marker.
// One 16-byte slot: the pair (a << 32 | b), how many rows hold it, and the first of them,
// so a lookup reads one slot; the factor sum is read only for a pair held by several rows.
struct alignas(16) PairSlot {
    uint64_t key;
    uint32_t cnt;
    uint32_t rid;
};
struct PairHash {
    PairSlot *slot;            // [cap + 1]
    uint64_t *msum;            // [cap + 1] sum of the rows' checksum factors
    uint32_t rel;              // relation the rows belong to (their checksum factors)
    uint32_t cap;              // power of two, >= 2 * rows + 1
    uint32_t *mask;            // device-side mask used (sized from the entry count)
    // membership bitmap in front of the table: 4 bits per slot in use (>= 8 per pair),
    // one bit per pair; a clear bit answers "absent" without touching the table
    uint32_t *sig;             // [cap / 8] words
    // bucket position of the pair's first row ([cap + 1]); with the rows sorted by pair,
    // the pair's rows are the bucket entries [pos, pos + count)
    uint32_t *pos;
};
// Fill `h` from n_dev entries: pair (ca[e], cb[e]), checksum factor of (rel, rid[e]).
hipError_t launch_pair_build(const PairHash &h, const uint32_t *n_dev, uint32_t cap_rows, const uint32_t *rid,
                             const int32_t *ca, const int32_t *cb, uint32_t rel, hipStream_t s);

constexpr uint32_t kTriBlocks = 2048;   // persistent grid of the intersection walk
struct TriArgs {
    // root survivors: x joins P's key, y joins L's closing column
    const uint32_t *n_root;
    uint32_t root_cap;
    const uint32_t *root_rid;
    const int32_t *root_x, *root_y;
    uint32_t rel_root;
    // P grouped by its key (x): directory and, per entry, row id and z (its key toward L)
    const uint64_t *P_slots;
    const uint32_t *P_mask, *P_begin, *P_rid;
    const int32_t *P_z;
    uint32_t rel_P;
    // L grouped by its closing column (y): directory and, per entry, row id and its key toward P
    const uint64_t *L_slots;
    const uint32_t *L_mask, *L_begin, *L_rid;
    const int32_t *L_z;
    uint32_t rel_L;
    PairHash HP;               // P's (x, z) pairs
    PairHash HL;               // L's (y, z) pairs
    uint32_t *w;               // [root_cap] walk length of each root entry | (walks L) << 31
    uint32_t *beg;             // [root_cap] first entry of the walked group
    uint64_t *off;             // [root_cap + 1] exclusive prefix of walk lengths
    uint64_t *tile_sums;       // [tiles(root_cap)]
    uint64_t *part;            // [2 * kTriBlocks] per-block count and checksum
    uint64_t *totals;          // [2] count, checksum
    // the write pass's offsets: the count pass writes each lane's and each workgroup's
    // tuple count (the write pass gives every lane the same walk steps)
    uint64_t *lane_cnt;        // [kTriBlocks * 256]
    uint64_t *block_cnt;       // [kTriBlocks]
};
hipError_t launch_tri_count(const TriArgs &a, hipStream_t s);

// 4-cliques by intersection: variables a, b (the root's two join columns), c and d; the
// other five relations each hold one of the pairs ac, ad, bc, bd, cd. Index h below:
// 0 ac, 1 ad, 2 bc, 3 bd, 4 cd.
struct K4Group {               // a relation grouped by its earlier variable (a, a, b, b, c)
    const uint64_t *slots;     // directory hash index: key -> directory entry
    const uint32_t *mask, *begin, *rid;
    const int32_t *other;      // per entry: the later variable (c, d, c, d, d)
    uint32_t rel;
};
struct K4Args {
    const uint32_t *n_root;
    uint32_t root_cap;
    const uint32_t *root_rid;
    const int32_t *root_a, *root_b;
    uint32_t rel_root;
    K4Group g[5];
    PairHash h[5];             // each relation's (earlier, later) pairs
    uint32_t *w;               // [root_cap] first-level walk length | (walks bc) << 31
    uint32_t *beg;             // [root_cap] first entry of the walked group
    uint64_t *off;             // [root_cap + 1] exclusive prefix of walk lengths
    uint64_t *tile_sums;       // [tiles(root_cap)]
    uint64_t *part;            // [2 * kTriBlocks]
    uint64_t *totals;          // [2] count, checksum
    uint64_t *lane_cnt;        // [kTriBlocks * 256] tuples of each lane (written by the count pass)
    uint64_t *block_cnt;       // [kTriBlocks] tuples of each workgroup
};
hipError_t launch_k4_count(const K4Args &a, hipStream_t s);

// Write pass of 3-cycles and 4-cliques by intersection: the count pass's walk again,
// once counting each lane's tuples and once writing them at the lane's offset (lanes
// in order, each lane's tuples in walk order). Roles: root, P, L (3-cycles) or root,
// ac, ad, bc, bd, cd (4-cliques).
struct CliqueOut {
    int32_t *out;              // [count, nrels] row ids in relation order, or [count, proj.n] values
    uint64_t capacity;         // tuples `out` holds (>= count; checked again per tuple)
    int nrels;
    Projection proj;           // proj.n == 0: row ids
    int role_rel[6];           // relation index of each role
    uint64_t *lane_cnt;        // [kTriBlocks * 256] tuples of each lane
    uint64_t *block_cnt;       // [kTriBlocks] tuples of each workgroup
};
constexpr uint32_t kEmitLanes = kTriBlocks * 256;
hipError_t launch_tri_emit(const TriArgs &a, const CliqueOut &o, hipStream_t s);
hipError_t launch_k4_emit(const K4Args &a, const CliqueOut &o, hipStream_t s);

}  // namespace sj
