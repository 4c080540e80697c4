// Alg. 4 (bottom-up construction with ropes, Sec. 4) run by host threads
// over std::atomic compare-and-swap, for ThreadSanitizer.  Test
// infrastructure: it checks the publish/read protocol of the box merge,
// not the GPU kernels (it shares no code with them).
//
// Protocol under test: a thread writes its node's box, then CASes the
// parent's `store` slot with release semantics; the second thread to
// arrive CASes with acquire semantics and only then reads its sibling's
// box.  With --racy the first thread publishes its box after the CAS (the
// wrong order), which ThreadSanitizer must report.
//
// stdin : n, then delta*[n-1] (ints, 255 = infinity), then the n leaf boxes
//         in sorted order (6 floats each: lo xyz, hi xyz).
// stdout: left[n-1], rope[2n-1], then 2n-1 boxes (unified ids: internal k
//         -> k, leaf k -> n-1+k, sentinel -1).
#include <algorithm>
#include <atomic>
#include <cstdio>
#include <cstring>
#include <random>
#include <thread>
#include <vector>

int main(int argc, char **argv)
{
    const bool racy = argc > 1 && std::strcmp(argv[1], "--racy") == 0;
    long n = 0;
    if (std::scanf("%ld", &n) != 1 || n < 1) return 2;
    std::vector<int> delta(n > 1 ? n - 1 : 0);
    for (auto &d : delta)
        if (std::scanf("%d", &d) != 1) return 2;
    const long total = 2 * n - 1, leaf0 = n - 1;
    std::vector<float> box(6 * total);
    for (long k = 0; k < n; ++k)
        for (int a = 0; a < 6; ++a)
            if (std::scanf("%f", &box[6 * (leaf0 + k) + a]) != 1) return 2;
    std::vector<int> left(n > 1 ? n - 1 : 0, -9), rope(total, -9);
    std::vector<std::atomic<int>> store(n > 1 ? n - 1 : 1);
    for (auto &s : store) s.store(-1, std::memory_order_relaxed);

    auto D = [&](long g) -> int { return (g < 0 || g >= n - 1) ? 255 : delta[g]; };

    auto climb = [&](long i) {
        long rl = i, rr = i, cur = leaf0 + i;
        int dl = D(i - 1), dr = D(i);
        rope[cur] = (i == n - 1) ? -1 : (dr < D(i + 1) ? (int)(leaf0 + i + 1) : (int)(i + 1));
        if (n == 1) return;
        // element-wise copies: a small memcpy is expanded inline by the
        // compiler and those stores are not seen by the sanitizer
        float own[6];
        for (int a = 0; a < 6; ++a) own[a] = box[6 * cur + a];
        auto publish = [&](long node) {
            for (int a = 0; a < 6; ++a) box[6 * node + a] = own[a];
        };
        bool unpublished = false;   // racy order: box[cur] not yet written
        while (true) {
            const bool is_left = dr < dl;
            const long p = is_left ? rr : rl - 1;
            int other = -1;
            const int mine = (int)(is_left ? rl : rr);
            // the correct order has published box[cur] before this CAS; the
            // racy order publishes an internal node's box only after it
            const bool first = store[p].compare_exchange_strong(
                other, mine, std::memory_order_acq_rel, std::memory_order_acquire);
            if (unpublished) publish(cur);
            if (first) return;   // first to arrive
            if (is_left) { rr = other; dr = D(rr); }
            else { rl = other; dl = D(rl - 1); }
            const long sib = is_left ? ((p + 1 == rr) ? leaf0 + p + 1 : p + 1)
                                     : ((rl == p) ? leaf0 + p : p);
            for (int a = 0; a < 3; ++a) {
                own[a] = std::min(own[a], box[6 * sib + a]);
                own[3 + a] = std::max(own[3 + a], box[6 * sib + 3 + a]);
            }
            const long q = dr < dl ? rr : rl;
            left[q] = (int)((rl == p) ? leaf0 + p : p);
            rope[q] = (rr == n - 1) ? -1 : (dr < D(rr + 1) ? (int)(leaf0 + rr + 1) : (int)(rr + 1));
            if (racy) unpublished = true;
            else publish(q);   // published before q's own CAS
            cur = q;
            if (q == 0) {
                if (unpublished) publish(cur);
                return;
            }
        }
    };

    // small trees: one thread per leaf, so a first arriver exits right
    // after its CAS and no later synchronisation of its can order a late
    // write before the sibling's read; larger trees: 8 threads
    const int T = n <= 256 ? (int)n : 8;
    // every thread waits until all exist: a thread that finished before
    // another was created would be ordered before it (thread start), which
    // would hide a late publication from the sanitizer
    std::atomic<int> ready{0};
    std::vector<std::thread> th;
    for (int t = 0; t < T; ++t)
        th.emplace_back([&, t] {
            ready.fetch_add(1, std::memory_order_relaxed);
            while (ready.load(std::memory_order_relaxed) < T) std::this_thread::yield();
            if (T == n) {   // one leaf, no allocation (a freed and reused
                climb(t);   // block would order threads for the sanitizer)
                return;
            }
            std::vector<long> mine;
            for (long i = t; i < n; i += T) mine.push_back(i);
            std::shuffle(mine.begin(), mine.end(), std::mt19937(1234 + t));
            for (long i : mine) {
                climb(i);
                if ((i & 7) == 0) std::this_thread::yield();
            }
        });
    for (auto &x : th) x.join();
    for (long k = 0; k + 1 < n; ++k) std::printf("%d\n", left[k]);
    for (long k = 0; k < total; ++k) std::printf("%d\n", rope[k]);
    for (long k = 0; k < total; ++k)
        for (int a = 0; a < 6; ++a) std::printf("%.9g\n", box[6 * k + a]);
    return 0;
}
