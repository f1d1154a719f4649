// Host planner of the persistent round kernel (see fbt_round.h for the task
// graph): the order in which the kernel's workgroups take the tasks.
#pragma once
#include <stdint.h>

#include <string>
#include <vector>

#include "fbt_round.h"

namespace fbt {

struct RPlanField {
    int64_t n; // observations
    int T;     // tiles of the bordered order
    int mode;  // 0 none, 1 Algorithm 2, 2 Algorithm 3
};

struct RPlan {
    std::vector<RTask> order;  // ticket order (queue after queue)
    std::vector<int64_t> qoff; // queue q holds order[qoff[q], qoff[q + 1])
    double est_us = 0.0;       // makespan of the list schedule under the cost model
    double busy_us = 0.0;      // sum of the task costs
};

// Ticket order of every task of the fields for `slots` workgroups taking
// tasks in that order: a list schedule (the ready task whose path to the end
// of its field is longest goes first) simulated under a cost model of tile
// size bt.  The order is checked with rplan_check before it is returned;
// on a failed check the result is empty and *err says why.
RPlan rplan(const std::vector<RPlanField> &fields, int bt, int slots, std::string *err);

// The fields split over nq queues (largest estimated work first, each to
// the queue with the least work so far), each queue planned by rplan for
// slots / nq workgroups: a queue's workgroups (one XCD's, in the kernel) then
// work on few fields at a time, whose tiles share that XCD's L2.
RPlan rplan_queues(const std::vector<RPlanField> &fields, int bt, int slots, int nq,
                   std::string *err);

// Executes `order` one task at a time on the counters (rdeps / rpublish):
// "" if every task finds its waits satisfied when its turn comes (so that
// workgroups taking tasks in this order can never wait on a task that no
// workgroup holds) and every task of every field occurs exactly once;
// otherwise the first violation.
std::string rplan_check(const std::vector<RTask> &order, const std::vector<RPlanField> &fields);

// Number of tasks of a field.
int64_t rtask_count(int T, int mode);

} // namespace fbt
