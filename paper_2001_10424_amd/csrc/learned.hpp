// Interface of the learned inner preconditioner (flexible CG whose
// preconditioner adds a CNN correction to one multigrid V-cycle, with plain
// multigrid-PCG as fallback).  Definitions live in learned_impl.hpp, which
// gkb.hip includes after the context type is complete.
#pragma once

struct gkb_ctx;
struct Learned;

namespace {
// learned_solve's return value when the network failed one of its guards:
// the caller runs the plain MG-PCG solve (from x = 0) instead
constexpr int kLearnedDeclined = 2;
bool learned_enabled(Learned* L);
bool learned_has_net(Learned* L);
bool learned_capturing(Learned* L);
void learned_reset(Learned* L);
template <typename T>
int learned_solve(gkb_ctx* c, const double* f, double* x_out, double tol, int* iters);
template <typename T>
int capture_solve(gkb_ctx* c, const double* f, double* x_out, double tol, int* iters);
int learned_create(gkb_ctx* c);
void learned_destroy(gkb_ctx* c);
}  // namespace
