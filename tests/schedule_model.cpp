// Host-thread model of the GPU library's two solve schedules (test only).
//
// Each "workgroup" of a GPU launch is a host thread; tile data are plain
// arrays and every flag, counter and queue is a std::atomic, so that
// ThreadSanitizer checks that every read of a tile is ordered after the write
// it needs (and every write after the reads it must not disturb).  The
// blocked Floyd-Warshall rounds (Section 2.3: phase 1 on the diagonal block,
// phases 2-3 on the row and column blocks, phase 4 on the rest; here phase 1,
// the bands, phase 3) run on int32 distances with successors, on tiles of
// T x T entries.
//
// Modelled, decision for decision:
//  - the persistent schedule (one launch): per-round queues (shared queue for
//    phase 1, the 2 nt band tiles and the next band's phase-3 tiles, then
//    eight XCD ranges), the epoch-valued flags diag, rowf/colf, nrow/ncol,
//    the counters done, p2c, rrd/crd, the ready3 shortcut (one acquire per
//    workgroup and round once every band tile is published), the forwarding
//    of band-K tiles that round K+1 reads, per-parity band maxima;
//  - the three-launch schedule with lookahead: on the caller's stream phase 3
//    of round K in two launches (the next band's tiles, then the rest), round
//    K+1's phases 1-2 on a second stream between two events, the direct-copy
//    phase 3 reading per-parity operand panels that the band tiles write, its
//    fix-up list, and launch boundaries as joins.
// A publish is a release store (the kernel: stores drained, barrier, an
// agent-scope release fence, then a relaxed store); a wait is a spin of
// acquire loads (the kernel: relaxed loads, then an agent-scope acquire
// fence).  Random delays between the steps vary the interleavings.
//
// Usage: schedule_model <sched: persistent|three> <n> <T> <grid> <seed> <reps> [mutation]
// Exit status 0 when every run matches the sequential blocked solve and the
// plain triple loop; 1 on a wrong result; 2 on a wait that never ends.
// The mutations plant one protocol mistake each (test of the model itself):
// persistent: no-war (band tiles skip the write-after-read counters), no-done
// (phase-3 tiles skip the previous round), ready3-any (the shortcut without
// all band tiles published), keep-ready3 (the shortcut carried into the next
// round), no-diag (band tiles skip phase 1); three launches: no-evb (phase 3
// does not wait for the next round's phases 1-2), no-eva (the second stream
// does not wait for the next band's tiles), one-parity (one set of operand
// panels).  Dropping the forwarder's wait (a band-K tile that round K+1
// reads) is not among them: the reader counters already imply it, since
// every counted reader acquired that tile.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <memory>
#include <random>
#include <string>
#include <thread>
#include <vector>

namespace {

constexpr uint32_t kInf = 1u << 30;
constexpr int kXcds = 8;

int n, T, nt, R;
std::string mut;
bool has(const char *m) { return mut == m; }

struct Mat {
    std::vector<uint32_t> D;
    std::vector<int32_t> NX;
};

thread_local std::mt19937 rng_tl;
void delay() {
    const uint32_t r = rng_tl() % 16;
    if (r < 8) return;
    if (r < 14) { std::this_thread::yield(); return; }
    std::this_thread::sleep_for(std::chrono::microseconds(rng_tl() % 60));
}

std::atomic<bool> g_hung{false};
bool spin_until(const std::atomic<int> &a, int v) {
    const auto t0 = std::chrono::steady_clock::now();
    while (a.load(std::memory_order_acquire) < v) {
        if (std::chrono::steady_clock::now() - t0 > std::chrono::seconds(30)) {
            g_hung = true;
            return false;
        }
        std::this_thread::yield();
    }
    return true;
}

// ---- tile arithmetic (the same product form and tie-break as the kernels)

int band_lo(int K) { return K * T; }
int band_hi(int K) { return std::min(n, K * T + T); }

// Where a tile of a launch lies: mode 0 remainder, 1 row band, 2 column band.
// False when every row or every column belongs to the band.
bool band_tile(int mode, int idx, int K, int &row0, int &col0) {
    const int b0 = band_lo(K), b1 = band_hi(K);
    if (mode == 0) { row0 = (idx / nt) * T; col0 = (idx % nt) * T; }
    else if (mode == 1) { row0 = b0; col0 = idx * T; }
    else { row0 = idx * T; col0 = b0; }
    if (mode != 1 && row0 >= b0 && std::min(row0 + T, n) <= b1) return false;
    if (mode != 2 && col0 >= b0 && std::min(col0 + T, n) <= b1) return false;
    return true;
}

void phase1(Mat &m, int K) {
    const int b0 = band_lo(K), b1 = band_hi(K);
    for (int k = b0; k < b1; ++k) {
        for (int i = b0; i < b1; ++i)
            for (int j = b0; j < b1; ++j) {
                const uint32_t s = m.D[(size_t)i * n + k] + m.D[(size_t)k * n + j];
                if (s < m.D[(size_t)i * n + j]) {
                    m.D[(size_t)i * n + j] = s;
                    m.NX[(size_t)i * n + j] = m.NX[(size_t)i * n + k];
                }
            }
        if ((k & 1) == 0) delay();
    }
}

// Operand panels of the direct-copy phase 3 (two round parities): A'[k][i]
// = D[i][b0 + k], B'[k][j] = D[b0 + k][j]; band maxima per parity.
struct Panels {
    std::vector<uint32_t> a[2], b[2];
    std::vector<uint32_t> bmax[2];   // row band tiles, then column band tiles
};

// C <- min(C, A (x) B) over the band of round K for one tile; A and B as the
// launch found them (the bands read their own old values).  With panels
// (direct-copy tile) the operands come from the panels instead of D.
void minplus(Mat &m, int K, int mode, int row0, int col0, Panels *pan, bool write_bmax, bool write_panel,
             bool read_panel, bool read_bmax) {
    const int b0 = band_lo(K), b1 = band_hi(K), bk = b1 - b0;
    const int r1 = (mode == 1) ? b1 : std::min(row0 + T, n);
    const int c1 = (mode == 2) ? b1 : std::min(col0 + T, n);
    const int rows = r1 - row0, cols = c1 - col0;
    const int par = has("one-parity") ? 0 : (K & 1);
    if (read_bmax) {
        // the phase-3 tile decides between packed keys and the general form
        // from the band maxima (the result is the same either way)
        volatile uint32_t ma = pan->bmax[par][nt + row0 / T], mb = pan->bmax[par][col0 / T];
        (void)ma; (void)mb;
    }
    std::vector<uint32_t> A((size_t)rows * bk), B((size_t)bk * cols), C((size_t)rows * cols);
    std::vector<int32_t> NA((size_t)rows * bk), NC((size_t)rows * cols);
    for (int i = 0; i < rows; ++i)
        for (int k = 0; k < bk; ++k) {
            A[(size_t)i * bk + k] = read_panel ? pan->a[par][(size_t)k * n + row0 + i]
                                               : m.D[(size_t)(row0 + i) * n + b0 + k];
        }
    delay();
    for (int k = 0; k < bk; ++k)
        for (int j = 0; j < cols; ++j)
            B[(size_t)k * cols + j] = read_panel ? pan->b[par][(size_t)k * n + col0 + j]
                                                 : m.D[(size_t)(b0 + k) * n + col0 + j];
    for (int i = 0; i < rows; ++i)
        for (int j = 0; j < cols; ++j) C[(size_t)i * cols + j] = m.D[(size_t)(row0 + i) * n + col0 + j];
    delay();
    // successors of A's entries (for the column band: the tile's own, old)
    for (int i = 0; i < rows; ++i)
        for (int k = 0; k < bk; ++k) NA[(size_t)i * bk + k] = m.NX[(size_t)(row0 + i) * n + b0 + k];
    std::vector<char> imp((size_t)rows * cols, 0);
    for (int i = 0; i < rows; ++i)
        for (int j = 0; j < cols; ++j) {
            uint32_t best = C[(size_t)i * cols + j];
            int kb = -1;
            for (int k = 0; k < bk; ++k) {
                const uint32_t s = A[(size_t)i * bk + k] + B[(size_t)k * cols + j];
                if (s < best) { best = s; kb = k; }
            }
            if (kb >= 0) {
                C[(size_t)i * cols + j] = best;
                NC[(size_t)i * cols + j] = NA[(size_t)i * bk + kb];
                imp[(size_t)i * cols + j] = 1;
            }
        }
    delay();
    for (int i = 0; i < rows; ++i)
        for (int j = 0; j < cols; ++j) {
            const int gi = row0 + i, gj = col0 + j;
            if (mode == 0 && ((gi >= b0 && gi < b1) || (gj >= b0 && gj < b1))) continue;
            if (mode == 1 && gj >= b0 && gj < b1) continue;
            if (mode == 2 && gi >= b0 && gi < b1) continue;
            if (!imp[(size_t)i * cols + j]) continue;      // only improved entries are stored
            m.D[(size_t)gi * n + gj] = C[(size_t)i * cols + j];
            m.NX[(size_t)gi * n + gj] = NC[(size_t)i * cols + j];
        }
    if ((write_panel || write_bmax) && mode != 0) {
        uint32_t mx = 0;
        for (int i = 0; i < rows; ++i)
            for (int j = 0; j < cols; ++j) {
                const uint32_t v = m.D[(size_t)(row0 + i) * n + col0 + j];
                if (v < kInf && v > mx) mx = v;
                if (!write_panel) continue;
                if (mode == 1) pan->b[par][(size_t)i * n + col0 + j] = v;
                else pan->a[par][(size_t)j * n + row0 + i] = v;
            }
        if (write_bmax) pan->bmax[par][(mode == 1 ? 0 : nt) + (mode == 1 ? col0 : row0) / T] = mx;
    }
}

void init(Mat &m, const std::vector<uint32_t> &W) {
    m.D.assign((size_t)n * n, 0);
    m.NX.assign((size_t)n * n, -1);
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) {
            const uint32_t w = (i == j) ? 0 : std::min(W[(size_t)i * n + j], kInf);
            m.D[(size_t)i * n + j] = w;
            m.NX[(size_t)i * n + j] = (i == j) ? i : (w < kInf ? j : -1);
        }
}

// ---- sequential references

void sequential_blocked(Mat &m) {
    for (int K = 0; K < R; ++K) {
        phase1(m, K);
        if (R == 1) break;
        for (int mode = 1; mode <= 2; ++mode)
            for (int q = 0; q < nt; ++q) {
                int r0, c0;
                if (band_tile(mode, q, K, r0, c0)) minplus(m, K, mode, r0, c0, nullptr, false, false, false, false);
            }
        for (int q = 0; q < nt * nt; ++q) {
            int r0, c0;
            if (band_tile(0, q, K, r0, c0)) minplus(m, K, 0, r0, c0, nullptr, false, false, false, false);
        }
    }
}

void triple_loop(std::vector<uint64_t> &D, const std::vector<uint32_t> &W) {
    D.assign((size_t)n * n, 0);
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) D[(size_t)i * n + j] = (i == j) ? 0 : std::min(W[(size_t)i * n + j], kInf);
    for (int k = 0; k < n; ++k)
        for (int i = 0; i < n; ++i)
            for (int j = 0; j < n; ++j) {
                const uint64_t s = D[(size_t)i * n + k] + D[(size_t)k * n + j];
                if (s < D[(size_t)i * n + j]) D[(size_t)i * n + j] = s;
            }
}

// ---- persistent schedule

using AtomArr = std::unique_ptr<std::atomic<int>[]>;
AtomArr zeros(size_t k) {
    AtomArr a(new std::atomic<int>[k]);
    for (size_t i = 0; i < k; ++i) a[i].store(0, std::memory_order_relaxed);
    return a;
}

struct PersistWs {
    std::atomic<int> diag{0};
    AtomArr q, xq, done, p2c, rrd, crd, rowf, colf, nrow, ncol;
    PersistWs() {
        q = zeros(R); xq = zeros((size_t)kXcds * R); done = zeros(R); p2c = zeros(R);
        rrd = zeros(R); crd = zeros(R);
        rowf = zeros(nt); colf = zeros(nt); nrow = zeros(nt); ncol = zeros(nt);
    }
};

// Phase-3 queue position q of round K -> tile (ti, tj); the next band's tiles
// (nxt = K + 1) come first.
void p3_tile(int64_t q, int nxt, int &ti, int &tj) {
    if (nxt >= nt) { ti = (int)(q / nt); tj = (int)(q % nt); return; }
    if (q == 0) { ti = tj = nxt; return; }
    q -= 1;
    if (q < nt - 1) { ti = nxt; tj = (int)(q < nxt ? q : q + 1); return; }
    q -= nt - 1;
    if (q < nt - 1) { tj = nxt; ti = (int)(q < nxt ? q : q + 1); return; }
    q -= nt - 1;
    const int a = (int)(q / (nt - 1)), b = (int)(q % (nt - 1));
    ti = a < nxt ? a : a + 1;
    tj = b < nxt ? b : b + 1;
}

void persistent_worker(Mat &m, PersistWs &ws, Panels &pan, int block, int seed) {
    rng_tl.seed(seed * 7919u + block);
    const int items = 1 + 2 * nt + nt * nt;
    const int xcd = block % kXcds;
    const int pq = (nt > 1) ? 2 * nt - 1 : 0;
    auto rel = std::memory_order_release;
    for (int K = 0; K < R; ++K) {
        const int pqk = (K + 1 < nt) ? pq : 0;
        const int lim0 = 1 + 2 * nt + pqk;
        const int rest = nt * nt - pqk;
        const int per = (rest + kXcds - 1) / kXcds;
        int mine = 0;
        static thread_local bool ready3 = false;
        if (!has("keep-ready3")) ready3 = false;
        int stage = 0;
        auto fetch = [&]() -> int {
            if (stage == 0) {
                const int v = ws.q[K].fetch_add(1, std::memory_order_relaxed);
                if (v < lim0) return v;
                stage = 1;
            }
            while (stage <= kXcds) {
                const int x = (xcd + stage - 1) % kXcds;
                const int tq = ws.xq[(size_t)K * kXcds + x].fetch_add(1, std::memory_order_relaxed);
                const int pos = pqk + x * per + tq;
                if (tq < per && pos < nt * nt) return 1 + 2 * nt + pos;
                ++stage;
            }
            return items;
        };
        int upcoming = fetch();
        for (;;) {
            const int item = upcoming;
            if (item >= items) break;
            ++mine;
            upcoming = fetch();
            delay();
            int mode = 0, ti = 0, tj = 0;
            if (item > 0 && item <= 2 * nt) {
                mode = item <= nt ? 1 : 2;
                ti = tj = (item - 1) % nt;
            } else if (item > 2 * nt) {
                p3_tile(item - 1 - 2 * nt, K + 1, ti, tj);
            }
            int row0 = 0, col0 = 0;
            const bool work = item > 0 && band_tile(mode, mode == 0 ? ti * nt + tj : ti, K, row0, col0);
            const bool feeds = item > 2 * nt && (ti == K + 1 || tj == K + 1);
            const bool waits = item <= 2 * nt || (work && !ready3) || (!work && feeds);
            if (waits) {
                int ok = 1;
                if (item == 0) {
                    ok = K == 0 || spin_until(ws.nrow[K], K);
                } else if (item <= 2 * nt) {
                    if (!has("no-diag")) ok = spin_until(ws.diag, K + 1);
                    if (ok && K > 0) ok = spin_until(mode == 1 ? ws.nrow[tj] : ws.ncol[ti], K);
                    if (ok && K > 0 && ti == K - 1 && !has("no-war"))
                        ok = spin_until(mode == 1 ? ws.rrd[K - 1] : ws.crd[K - 1], nt - 1);
                } else if (work) {
                    if (!has("no-done")) ok = K == 0 || spin_until(ws.done[K - 1], items);
                    const bool all2 = ok && ws.p2c[K].load(std::memory_order_acquire) >= 2 * nt;
                    if (ok && !all2) ok = spin_until(ws.rowf[tj], K + 1) && spin_until(ws.colf[ti], K + 1);
                    if (ok && (all2 || has("ready3-any"))) ok = 2;
                } else {
                    ok = (ti == K) ? spin_until(ws.rowf[tj], K + 1) : spin_until(ws.colf[ti], K + 1);
                }
                if (!ok) return;
                if (item > 2 * nt && work && ok == 2) ready3 = true;
            }
            delay();
            if (item == 0) phase1(m, K);
            else if (work) minplus(m, K, mode, row0, col0, &pan, mode != 0, false, false, mode == 0);
            delay();
            if (item == 0) {
                ws.diag.store(K + 1, rel);
            } else if (item <= 2 * nt) {
                (mode == 1 ? ws.rowf[tj] : ws.colf[ti]).store(K + 1, rel);
                ws.p2c[K].fetch_add(1, rel);
            } else if (feeds) {
                if (ti == K + 1) ws.nrow[tj].store(K + 1, rel);
                if (tj == K + 1) ws.ncol[ti].store(K + 1, rel);
                if (work) {
                    if (ti == K + 1) ws.rrd[K].fetch_add(1, rel);
                    if (tj == K + 1) ws.crd[K].fetch_add(1, rel);
                }
            }
        }
        ws.done[K].fetch_add(mine, rel);
    }
}

// ---- three launches per round, lookahead on a second stream

// A launch: its tiles run on `grid` threads in a random order; the launch
// ends when every thread has joined (the kernel boundary).
template <typename F>
void launch(int ntiles, int grid, int seed, F body) {
    if (ntiles <= 0) return;
    std::vector<int> order(ntiles);
    for (int i = 0; i < ntiles; ++i) order[i] = i;
    std::mt19937 g(seed);
    std::shuffle(order.begin(), order.end(), g);
    std::atomic<int> next{0};
    std::vector<std::thread> th;
    const int w = std::max(1, std::min(grid, ntiles));
    for (int b = 0; b < w; ++b)
        th.emplace_back([&, b] {
            rng_tl.seed(seed * 31u + b);
            for (;;) {
                const int q = next.fetch_add(1, std::memory_order_relaxed);
                if (q >= ntiles) break;
                delay();
                body(order[q]);
            }
        });
    for (auto &t : th) t.join();
}

// Tile of a phase-3 launch: part 1 = the next band's tiles, part 2 = the rest,
// part 0 = all (the kernels' mapping; -1 = none).
int phase3_tile_of(int part, int q, int K) {
    if (part == 1) {
        const int nx1 = K + 1;
        if (q < nt) return nx1 * nt + q;
        if (q - nt == nx1) return -1;
        return (q - nt) * nt + nx1;
    }
    if (part == 2 && (q / nt == K + 1 || q % nt == K + 1)) return -1;
    return q;
}

struct Event {
    std::atomic<int> epoch{0};
    void record(int v) { epoch.store(v, std::memory_order_release); }
    bool wait(int v) { return spin_until(epoch, v); }
};

void three_launch(Mat &m, Panels &pan, int grid, int seed, bool direct) {
    // launch counters (seeds of the launches' tile orders), one per stream
    int ln_main = 0, ln_aux = 500000;
    auto p1 = [&](int K, int &ln) { launch(1, 1, seed + 1000 * ++ln, [&](int) { phase1(m, K); }); };
    auto p2 = [&](int K, int &ln) {
        launch(2 * nt, grid, seed + 1000 * ++ln, [&](int q) {
            const int mode = q < nt ? 1 : 2;
            int r0, c0;
            if (band_tile(mode, q % nt, K, r0, c0)) minplus(m, K, mode, r0, c0, &pan, true, direct, false, false);
        });
    };
    // the direct-copy phase 3: full tiles from the panels, the others to the
    // fix-up list, run afterwards by the general tile
    auto p3 = [&](int K, int part, int &ln) {
        const int cnt = part == 1 ? 2 * nt : nt * nt;
        std::vector<int> fix;
        std::atomic<int> nfix{0};
        fix.assign((size_t)nt * nt, -1);
        launch(cnt, grid, seed + 1000 * ++ln, [&](int q) {
            const int idx = phase3_tile_of(part, q, K);
            if (idx < 0) return;
            int r0, c0;
            if (!band_tile(0, idx, K, r0, c0)) return;
            const bool full = r0 + T <= n && c0 + T <= n && band_hi(K) - band_lo(K) == T;
            if (direct && full) minplus(m, K, 0, r0, c0, &pan, false, false, true, true);
            else if (direct) fix[nfix.fetch_add(1, std::memory_order_relaxed)] = idx;
            else minplus(m, K, 0, r0, c0, &pan, false, false, false, true);
        });
        const int nf = nfix.load(std::memory_order_relaxed);
        launch(nf, grid, seed + 1000 * ++ln, [&](int q) {
            int r0, c0;
            if (band_tile(0, fix[q], K, r0, c0)) minplus(m, K, 0, r0, c0, &pan, false, false, false, true);
        });
    };
    const bool ahead = R >= 3;
    if (!ahead) {
        for (int K = 0; K < R; ++K) {
            p1(K, ln_main);
            if (R == 1) break;
            p2(K, ln_main);
            p3(K, 0, ln_main);
        }
        return;
    }
    Event ev_a, ev_b;
    std::thread aux([&] {
        for (int K = 0; K + 1 < R; ++K) {
            if (!has("no-eva") && !ev_a.wait(K + 1)) return;
            p1(K + 1, ln_aux);
            p2(K + 1, ln_aux);
            ev_b.record(K + 1);
        }
    });
    p1(0, ln_main);
    p2(0, ln_main);
    for (int K = 0; K < R; ++K) {
        if (K + 1 == R) {
            p3(K, 0, ln_main);
            break;
        }
        p3(K, 1, ln_main);
        ev_a.record(K + 1);
        p3(K, 2, ln_main);
        if (!has("no-evb") && !ev_b.wait(K + 1)) break;
    }
    aux.join();
}

}  // namespace

int main(int argc, char **argv) {
    if (argc < 7) {
        fprintf(stderr, "usage: %s persistent|three n T grid seed reps [mutation]\n", argv[0]);
        return 64;
    }
    const std::string sched = argv[1];
    n = atoi(argv[2]);
    T = atoi(argv[3]);
    const int grid = atoi(argv[4]);
    const int seed = atoi(argv[5]);
    const int reps = atoi(argv[6]);
    if (argc > 7) mut = argv[7];
    nt = (n + T - 1) / T;
    R = nt;
    // input: edge probability 0.5, weights 1..9 (many ties), absent 2^30
    std::mt19937 g(seed);
    std::vector<uint32_t> W((size_t)n * n);
    for (auto &w : W) w = (g() % 2) ? 1 + g() % 9 : kInf;
    Mat ref;
    init(ref, W);
    sequential_blocked(ref);
    std::vector<uint64_t> tl;
    triple_loop(tl, W);
    for (size_t e = 0; e < tl.size(); ++e)
        if ((uint64_t)ref.D[e] != tl[e]) {
            fprintf(stderr, "sequential blocked solve differs from the triple loop at %zu\n", e);
            return 1;
        }
    for (int rep = 0; rep < reps; ++rep) {
        Mat m;
        init(m, W);
        Panels pan;
        for (int p = 0; p < 2; ++p) {
            pan.a[p].assign((size_t)T * n, 0);
            pan.b[p].assign((size_t)T * n, 0);
            pan.bmax[p].assign((size_t)2 * nt, 0);
        }
        if (sched == "persistent") {
            PersistWs ws;
            const int items = 1 + 2 * nt + nt * nt;
            const int gsz = std::max(1, std::min(grid, items));
            std::vector<std::thread> th;
            for (int b = 0; b < gsz; ++b)
                th.emplace_back([&, b] { persistent_worker(m, ws, pan, b, seed * 100 + rep); });
            for (auto &t : th) t.join();
        } else {
            three_launch(m, pan, grid, seed * 100 + rep, sched == "three");
        }
        if (g_hung) {
            fprintf(stderr, "a wait never ended (sched %s n %d T %d grid %d seed %d rep %d)\n", sched.c_str(), n,
                    T, grid, seed, rep);
            return 2;
        }
        for (size_t e = 0; e < m.D.size(); ++e)
            if (m.D[e] != ref.D[e] || m.NX[e] != ref.NX[e]) {
                fprintf(stderr, "wrong result at (%zu, %zu): D %u vs %u, NX %d vs %d (sched %s n %d T %d grid %d "
                        "seed %d rep %d)\n", e / n, e % n, m.D[e], ref.D[e], m.NX[e], ref.NX[e], sched.c_str(),
                        n, T, grid, seed, rep);
                return 1;
            }
    }
    printf("ok %s n=%d T=%d grid=%d seed=%d reps=%d\n", sched.c_str(), n, T, grid, seed, reps);
    return 0;
}
