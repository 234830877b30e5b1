// Batch planning helpers shared by the batched entry points (internal).
#pragma once
#include "ctx.hpp"

namespace gevd {

// Compute units of the handle's device (cached in the handle).
int batch_num_cu(gevd_ctx* h);
// Launch shape of a (scalar type, order bucket): the handle's table entry,
// else the occupancy-derived default.
void batch_shape_of(gevd_ctx* h, bool cx, int bucket, int* threads, int* wgpcu);
// 0 when the descriptor is valid for the batched path, else 1.
int batch_check_problem(const gevd_problem& p);
// Queue order of a batch written to ord[0..count): complex problems first
// (their group is the longer one), then decreasing order n, then input
// position.  In place, no allocation.
void batch_order(int count, const gevd_problem* probs, int* ord);
// Algorithmic flops of one problem (real count, x4 complex).
double batch_problem_flops(const gevd_problem& p);

// Resolves the device address of the fixed no-allocation scratch array on
// `device` (which must be current); called once per device from gevd_create.
int noalloc_attach(int device);

}  // namespace gevd
