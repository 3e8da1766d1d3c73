// Host-side planning of the all-pairs sweeps and the autotuning table that
// picks a sweep variant (rows per thread, waves per SIMD) per size class.
//
// Size class = floor(log2(n)) of the number of records of a single layout,
// or of the mean number of records per layout of a batch.  The table starts
// from built-in defaults, is updated by rb_autotune / rb_batch_autotune, and
// can be saved to and loaded from a text file ("kind batch class variant"
// per line).  RB_TUNE_CACHE names a file loaded on first use.
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>

#include "rb_internal.h"

namespace rb {

SweepLayout sweep_layout(int64_t n_items, int rows, int64_t unit_off, int64_t rec_off,
                         int col_shift) {
    const int64_t R = (int64_t)kBlock * rows;
    const int64_t W = (int64_t)(kChunk >> col_shift);
    const int64_t n = n_items > 0 ? n_items : 1;
    SweepLayout l;
    l.unit_off = unit_off;
    l.rec_off = rec_off;
    l.n_row_tiles = (n + R - 1) / R;
    l.n_chunks = (n + W - 1) / W;
    l.col_shift = col_shift;
    return l;
}

int64_t sweep_units(int64_t n_items, int rows, int col_shift) {
    const SweepLayout l = sweep_layout(n_items, rows, 0, 0, col_shift);
    return l.n_row_tiles * l.n_chunks -
           ((int64_t)rows << col_shift) * l.n_row_tiles * (l.n_row_tiles - 1) / 2;
}

namespace {

constexpr int kClasses = 40;
constexpr int kKinds = 4;   // 0 crossing, 1 crossing + angle, 2 occlusion, 3 pruned crossing
constexpr int kDefault[kKinds] = {1, 1, 2, 0};

struct Table {
    std::mutex mu;
    bool init = false;
    int v[kKinds][2][kClasses];
} g_tab;

int size_class(int64_t n) {
    int c = 0;
    while (n > 1 && c < kClasses - 1) {
        n >>= 1;
        ++c;
    }
    return c;
}

int n_variants(int kind) { return kind == 2 ? kOcclVariants : kCrossVariants; }

void load_locked(const char *path) {
    FILE *f = fopen(path, "r");
    if (!f) return;
    int kind, batch, cls, var;
    while (fscanf(f, "%d %d %d %d", &kind, &batch, &cls, &var) == 4) {
        if (kind >= 0 && kind < kKinds && (batch == 0 || batch == 1) && cls >= 0 &&
            cls < kClasses && var >= 0 && var < n_variants(kind) &&
            variant_offered(kind, batch != 0, var))
            g_tab.v[kind][batch][cls] = var;
    }
    fclose(f);
}

// the built-in default of a kind, batch flag and size class: the crossing
// sweeps take 2 rows per thread, and the crossing + angle sweep of a single
// layout 3 rows from 2^21 edges (0.7% faster than 2 rows and 1.4% than 4 at
// 3M edges); the pruned
// sweep takes the 1-row tiles (tightest boxes) below 2^17 edges and 2-row
// tiles above.  The node sweep of a single layout splits its 256-column
// chunks below 2^16 nodes, for units enough to fill the chip: 2 rows per
// thread and 32 columns below 2^13 nodes, 4 rows at 8 waves per SIMD and 32
// columns below 2^14, the same with 64 columns below 2^16 (two units per
// block from 2^15), and whole chunks at 4 rows and 8 waves from there.  A batch has units enough in any case
// and keeps 4-row tiles at 8 waves up to a mean of 2^19 nodes per layout.
int default_variant(int k, int b, int c) {
    if (k == 3 && c >= 17) return 1;
    if (k == 1 && !b && c >= 21) return 2;
    if (k == 2) {
        if (b) return c >= 19 ? 0 : 9;
        if (c <= 12) return 6;
        if (c == 13) return 11;
        if (c == 14 || c == 15) return 10;
        return 9;
    }
    return kDefault[k];
}

void defaults_locked() {
    for (int k = 0; k < kKinds; ++k)
        for (int b = 0; b < 2; ++b)
            for (int c = 0; c < kClasses; ++c) g_tab.v[k][b][c] = default_variant(k, b, c);
}

void init_locked() {
    if (g_tab.init) return;
    defaults_locked();
    g_tab.init = true;
    const char *path = getenv("RB_TUNE_CACHE");
    if (path && *path) load_locked(path);
}

}  // namespace

int tuned_variant(int kind, bool batch, int64_t n) {
    std::lock_guard<std::mutex> g(g_tab.mu);
    init_locked();
    return g_tab.v[kind][batch ? 1 : 0][size_class(n)];
}

void set_tuned_variant(int kind, bool batch, int64_t n, int variant) {
    std::lock_guard<std::mutex> g(g_tab.mu);
    init_locked();
    g_tab.v[kind][batch ? 1 : 0][size_class(n)] = variant;
}

bool save_tuning(const char *path) {
    std::lock_guard<std::mutex> g(g_tab.mu);
    init_locked();
    FILE *f = fopen(path, "w");
    if (!f) return false;
    for (int k = 0; k < kKinds; ++k)
        for (int b = 0; b < 2; ++b)
            for (int c = 0; c < kClasses; ++c)
                if (g_tab.v[k][b][c] != default_variant(k, b, c))
                    fprintf(f, "%d %d %d %d\n", k, b, c, g_tab.v[k][b][c]);
    return fclose(f) == 0;
}

bool load_tuning(const char *path) {
    std::lock_guard<std::mutex> g(g_tab.mu);
    init_locked();
    FILE *f = fopen(path, "r");
    if (!f) return false;
    fclose(f);
    defaults_locked();
    load_locked(path);
    return true;
}

}  // namespace rb
