// Learned inner preconditioner: definitions (included by gkb.hip).
#pragma once

struct Learned {
  bool enabled = false;
};

namespace {
bool learned_enabled(Learned* L) { return L && L->enabled; }
template <typename T>
int learned_solve(gkb_ctx*, const double*, double*, double, int*) { return GKB_EINVAL; }
int learned_create(gkb_ctx* c) {
  c->learned = new Learned();
  return GKB_OK;
}
void learned_destroy(gkb_ctx* c) {
  delete c->learned;
  c->learned = nullptr;
}
}  // namespace
