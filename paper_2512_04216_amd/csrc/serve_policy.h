// serve_policy.h -- admission policy of the request server (host only, no HIP).
//
// Requests wait in arrival order. One pass over the head of the queue
// (at most `lookahead` entries) decides, for each request:
//   * small (packed) requests are admitted while fewer than `max_small` wait for
//     a packed launch;
//   * a large request whose footprint exceeds the whole budget is rejected;
//   * a large request is admitted if a resident slot is free (fewer than
//     `max_large` resident) and the caller's allocator can place it (`fits`);
//   * otherwise it waits. Later requests may overtake a waiting head, but each
//     overtaking counts against the head; once the head has been overtaken
//     `max_bypass` times, nothing behind it is admitted until it fits.
#pragma once

#include <cstddef>
#include <cstdint>
#include <utility>
#include <vector>

namespace svp {

using std::size_t;

struct Candidate {
    bool small = false;
    uint64_t footprint = 0;   // bytes a large request holds while resident
    int bypassed = 0;         // times it was overtaken while at the head
};

enum class Action { AdmitSmall, AdmitLarge, Reject };

struct Limits {
    uint64_t budget = 0;      // bytes all resident large requests may hold
    int max_large = 256;      // resident large requests
    int max_small = 8192;     // small requests admitted but not yet launched
    int max_bypass = 32;
    int lookahead = 256;
};

// `fits(i)` tries to reserve what queue[i] needs and returns true on success
// (it is called only for large requests that pass the budget and slot checks).
// Returns (queue index, action) in the order taken; queue[0].bypassed is updated.
template <class Fits>
std::vector<std::pair<size_t, Action>> plan_admission(std::vector<Candidate> &queue, const Limits &lim,
                                                      uint64_t held, int nlarge, int nsmall, Fits fits) {
    std::vector<std::pair<size_t, Action>> out;
    const size_t n = queue.size() < (size_t)lim.lookahead ? queue.size() : (size_t)lim.lookahead;
    bool head_waiting = false;   // queue[0] is a large request that could not be admitted
    for (size_t i = 0; i < n; ++i) {
        Candidate &c = queue[i];
        if (head_waiting && queue[0].bypassed >= lim.max_bypass) break;
        if (c.small) {
            if (nsmall >= lim.max_small) continue;
            out.emplace_back(i, Action::AdmitSmall);
            ++nsmall;
            if (head_waiting) queue[0].bypassed++;
            continue;
        }
        if (c.footprint > lim.budget) {
            out.emplace_back(i, Action::Reject);
            continue;
        }
        if (nlarge < lim.max_large && held + c.footprint <= lim.budget && fits(i)) {
            out.emplace_back(i, Action::AdmitLarge);
            held += c.footprint;
            ++nlarge;
            if (head_waiting) queue[0].bypassed++;
            continue;
        }
        if (i == 0) head_waiting = true;
    }
    return out;
}

}  // namespace svp
