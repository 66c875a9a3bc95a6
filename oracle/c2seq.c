/* Sequential C statement of the release/admit rounds of the admission
 * microbenchmark -- CPU oracle, TEST INFRASTRUCTURE ONLY.
 *
 * Paper: Sec. V, Policy 1 (FIFO: serve waiting clients in order while each
 * fits the free memory; the first that does not fit stops the walk) and
 * Policy 2 (MMU: a client that does not fit keeps waiting and the walk goes
 * on with the next); Sec. IV post-free (a client returns what it holds);
 * Sec. III-B (free memory = total minus the reservations in use).
 *
 * This is the same computation as oracle/sched.py release_rounds, written as
 * the plain sequential loop a C programmer would write: the waiting requests
 * are a singly linked list in arrival order, the running jobs an array.  It
 * exists to time the oracle as compiled code on one host core; it shares no
 * code with the HIP library and is never called by it.
 *
 * Job j is queue position j.  Round 0 is one pass over the whole queue; in
 * round r >= 1 every running job j with coins[(r - 1) * n + j] != 0 releases
 * its whole reservation, then one pass runs.  A negative demand is a
 * withdrawn request: never admitted, never blocking.
 */
#include <stdint.h>
#include <stdlib.h>

/* Outputs per round r: adm_count[r] admitted ids appended to adm_ids (queue
 * order within a round), R_after[r] the free memory after the pass,
 * rel_count[r] jobs released before it.  adm_ids holds at least n entries.
 * Returns 0, or -1 for bad arguments or when memory cannot be had. */
int c2seq_release_rounds(int64_t n, const int64_t *demand, int64_t capacity,
                         const uint8_t *coins, int32_t rounds, int32_t policy,
                         int64_t *adm_count, int64_t *R_after, int64_t *rel_count,
                         int64_t *adm_ids) {
  if (n < 0 || rounds < 0 || capacity < 0 || (policy != 0 && policy != 1)) return -1;
  int64_t *next = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
  int64_t *run = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
  if (!next || !run) {
    free(next);
    free(run);
    return -1;
  }
  /* intake: every request waits, in arrival order */
  for (int64_t i = 0; i < n; ++i) next[i] = i + 1 < n ? i + 1 : -1;
  int64_t head = n > 0 ? 0 : -1;
  int64_t n_run = 0, used = 0, n_adm = 0;
  for (int32_t r = 0; r < rounds; ++r) {
    int64_t released = 0;
    if (r > 0) { /* post-free of every coin-chosen running job */
      const uint8_t *coin = coins + (int64_t)(r - 1) * n;
      int64_t keep = 0;
      for (int64_t k = 0; k < n_run; ++k) {
        const int64_t j = run[k];
        if (coin[j]) {
          used -= demand[j];
          ++released;
        } else {
          run[keep++] = j;
        }
      }
      n_run = keep;
    }
    int64_t R = capacity - used;
    int64_t got = 0;
    int64_t prev = -1, i = head;
    while (i >= 0) {
      if (policy == 1 && R == 0) break; /* every present demand is >= 1 */
      const int64_t nx = next[i];
      const int64_t d = demand[i];
      if (d >= 0 && d <= R) { /* admit: leaves the waiting list */
        R -= d;
        adm_ids[n_adm++] = i;
        run[n_run++] = i;
        ++got;
        if (prev < 0)
          head = nx;
        else
          next[prev] = nx;
      } else {
        if (policy == 0 && d >= 0) break; /* FIFO: the first misfit stops */
        prev = i;
      }
      i = nx;
    }
    used = capacity - R;
    adm_count[r] = got;
    R_after[r] = R;
    rel_count[r] = released;
  }
  free(next);
  free(run);
  return 0;
}
