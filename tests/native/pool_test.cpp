// Host-only checks of the workspace pool's return rule (compiled with g++).
#include <cstdio>
#include <cstdlib>

#include "pool.h"

#define EXPECT(c)                                                    \
  do {                                                               \
    if (!(c)) {                                                      \
      std::fprintf(stderr, "FAILED %s at line %d\n", #c, __LINE__);  \
      std::exit(1);                                                  \
    }                                                                \
  } while (0)

struct Fake {
  int id;
  int done;       // last device state
  bool failed;    // host guard
};

int main() {
  using reco::ReusePool;
  using reco::workspace_reusable;
  // the rule
  EXPECT(workspace_reusable(0, false, false));
  EXPECT(workspace_reusable(1, false, false));   // converged
  EXPECT(workspace_reusable(2, false, false));   // iteration cap
  EXPECT(workspace_reusable(3, false, false));   // non-finite scalars: buffers are consistent
  EXPECT(!workspace_reusable(4, false, false));  // a reduction gave up waiting
  EXPECT(!workspace_reusable(1, true, false));   // host guard tripped
  EXPECT(!workspace_reusable(1, false, true));   // ended in an exception

  ReusePool<Fake> pool;
  int dropped = 0;
  auto drop = [&](Fake* p) { ++dropped; delete p; };
  EXPECT(pool.take() == nullptr);
  Fake* a = new Fake{1, 1, false};
  Fake* b = new Fake{2, 4, false};
  Fake* c = new Fake{3, 2, true};
  EXPECT(pool.give_back(a, workspace_reusable(a->done, a->failed, false), drop));
  EXPECT(!pool.give_back(b, workspace_reusable(b->done, b->failed, false), drop));
  EXPECT(!pool.give_back(c, workspace_reusable(c->done, c->failed, false), drop));
  EXPECT(dropped == 2);
  EXPECT(pool.size() == 1);
  // only the clean workspace comes back out
  Fake* t = pool.take();
  EXPECT(t == a);
  EXPECT(pool.take() == nullptr);
  EXPECT(!pool.give_back(static_cast<Fake*>(nullptr), true, drop));
  EXPECT(pool.give_back(t, true, drop));
  EXPECT(pool.give_back(new Fake{4, 1, false}, true, drop));
  EXPECT(pool.drain(drop) == 2);
  EXPECT(dropped == 4);
  EXPECT(pool.size() == 0);
  std::printf("pool ok\n");
  return 0;
}
