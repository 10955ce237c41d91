// Host-only run of the server's scheduler (paper_2407_14783_amd/csrc/batcher.h) against a fake backend:
// batches "step" a host table of env states (x <- x / 2 + a, so the order of requests on one slot
// matters), finish after a random number of polls, and fail at random or by host-forced injection.
// Prints one JSON object with the checks' figures; tests/test_sched_host.py compiles and runs it.
//
// usage: sched_fake_backend <seed> <n_requests> <fail_prob> <inject> <max_attempts>
#include <cstdio>
#include <cstdlib>
#include <map>
#include <random>
#include <set>
#include <string>
#include <vector>

#include "batcher.h"

using vf::sched::Item;

struct Req : Item {
    int id = 0;
    std::vector<double> act;       // one action per env
    std::vector<double> result;    // the env states after the request's step
    int completions = 0;
};

struct Fake {
    std::vector<double> state;
    std::mt19937_64 rng;
    double fail_prob = 0.0;
    struct Flight {
        std::vector<Item*> items;
        std::vector<std::pair<int32_t, double>> snapshot;
        int polls_left = 0;
        bool doomed = false;
    };
    std::map<int, Flight> flight;
    std::multiset<int32_t> in_flight_slots;
    int64_t arena_bytes = 0;
    // figures for the checks
    int64_t overlap_violations = 0, budget_violations = 0, launches = 0, random_failures = 0;
    std::vector<int> completion_order;

    bool launch(int i, std::vector<Item*>& items) {
        Flight f;
        int64_t bytes = 0;
        for (Item* it : items) {
            bytes += it->bytes;
            for (int32_t sl : it->slots) {
                if (in_flight_slots.count(sl)) ++overlap_violations;
                in_flight_slots.insert(sl);
                f.snapshot.push_back({sl, state[sl]});
            }
        }
        if (bytes > arena_bytes) ++budget_violations;
        // the batch steps its envs now; a failure reported later leaves these changes for restore() to undo
        for (Item* it : items) {
            Req* r = static_cast<Req*>(it);
            for (size_t e = 0; e < r->slots.size(); ++e) state[r->slots[e]] = state[r->slots[e]] * 0.5 + r->act[e];
        }
        f.items = items;
        f.polls_left = (int)(rng() % 4);
        f.doomed = std::uniform_real_distribution<double>(0.0, 1.0)(rng) < fail_prob;
        flight[i] = f;
        ++launches;
        return true;
    }
    int poll(int i) {
        Flight& f = flight[i];
        if (f.polls_left-- > 0) return 0;
        if (f.doomed) {
            ++random_failures;
            return -1;
        }
        return 1;
    }
    void drop(int i) {
        for (Item* it : flight[i].items)
            for (int32_t sl : it->slots) in_flight_slots.erase(in_flight_slots.find(sl));
        flight.erase(i);
    }
    uint32_t finish(int i, std::vector<Item*>& items) {
        for (Item* it : items) {
            Req* r = static_cast<Req*>(it);
            r->result.clear();
            for (int32_t sl : r->slots) r->result.push_back(state[sl]);
        }
        drop(i);
        return 0;
    }
    bool restore(int i, std::vector<Item*>&) {
        Flight& f = flight[i];
        for (auto it = f.snapshot.rbegin(); it != f.snapshot.rend(); ++it) state[it->first] = it->second;
        drop(i);
        return true;
    }
    void on_done(Item* it) {
        Req* r = static_cast<Req*>(it);
        ++r->completions;
        completion_order.push_back(r->id);
    }
};

int main(int argc, char** argv) {
    if (argc < 6) return 2;
    const unsigned seed = (unsigned)atoi(argv[1]);
    const int n_req = atoi(argv[2]);
    const double fail_prob = atof(argv[3]);
    const int inject = atoi(argv[4]);
    const int max_attempts = atoi(argv[5]);
    const int n_slots = 64, n_arenas = 3;
    const int64_t arena_bytes = 40, max_batch = 24;
    std::mt19937_64 gen(seed);
    Fake fk;
    fk.rng.seed(seed * 7919u + 1u);
    fk.fail_prob = fail_prob;
    fk.arena_bytes = arena_bytes;
    fk.state.resize(n_slots);
    for (int k = 0; k < n_slots; ++k) fk.state[k] = k;
    std::vector<double> init = fk.state;
    vf::sched::Scheduler<Fake> sch(fk, n_arenas, arena_bytes, max_batch, max_attempts);
    sch.inject_faults(inject);
    std::vector<Req*> reqs;
    for (int q = 0; q < n_req; ++q) {
        Req* r = new Req();
        r->id = q;
        const int n_env = 1 + (int)(gen() % 8);
        std::set<int32_t> s;
        while ((int)s.size() < n_env) s.insert((int32_t)(gen() % n_slots));
        r->slots.assign(s.begin(), s.end());
        r->n_env = n_env;
        r->bytes = 4 + 3 * n_env;          // at most 28 of the arena's 40
        for (int e = 0; e < n_env; ++e) r->act.push_back((double)(gen() % 1000) / 7.0);
        reqs.push_back(r);
    }
    // requests arrive in bursts between scheduler passes
    size_t next = 0;
    int64_t passes = 0;
    while (next < reqs.size() || !sch.idle()) {
        const int burst = (int)(gen() % 5);
        for (int k = 0; k < burst && next < reqs.size(); ++k) sch.submit(reqs[next++]);
        sch.step();
        if (++passes > 10000000) break;
    }
    // the serial reference: every request that completed OK, in arrival order, one slot at a time
    std::vector<double> ref = init;
    int64_t ok = 0, failed = 0, wrong_results = 0, multi = 0, unfinished = 0;
    for (Req* r : reqs) {
        if (!r->done) {
            ++unfinished;
            continue;
        }
        if (r->completions != 1) ++multi;
        if (r->status != vf::sched::kOk) {
            ++failed;
            continue;
        }
        ++ok;
        for (size_t e = 0; e < r->slots.size(); ++e) {
            ref[r->slots[e]] = ref[r->slots[e]] * 0.5 + r->act[e];
            if (r->result.size() != r->slots.size() || r->result[e] != ref[r->slots[e]]) ++wrong_results;
        }
    }
    int64_t state_mismatch = 0;
    for (int k = 0; k < n_slots; ++k) state_mismatch += fk.state[k] != ref[k] ? 1 : 0;
    const auto& st = sch.stats();
    printf("{\"requests\": %d, \"ok\": %lld, \"failed\": %lld, \"unfinished\": %lld, \"completed_more_than_once\": %lld, "
           "\"wrong_results\": %lld, \"state_mismatch\": %lld, \"overlap_violations\": %lld, \"budget_violations\": %lld, "
           "\"batches\": %lld, \"failed_batches\": %lld, \"requeued\": %lld, \"random_failures\": %lld, "
           "\"launches\": %lld, \"max_batch\": %lld}\n",
           n_req, (long long)ok, (long long)failed, (long long)unfinished, (long long)multi, (long long)wrong_results,
           (long long)state_mismatch, (long long)fk.overlap_violations, (long long)fk.budget_violations,
           (long long)st.batches, (long long)st.failed_batches, (long long)st.requeued, (long long)fk.random_failures,
           (long long)fk.launches, (long long)st.max_batch);
    for (Req* r : reqs) delete r;
    return 0;
}
