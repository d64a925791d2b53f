// Batched timestep programs (program.cpp): cache management.
#pragma once

namespace stl {

// Releases cached graphs, plans and scratch of stencil_program_run.
void program_release_all();

// Device bytes held by cached programs; *programs (if given) receives the
// number of cached programs.
long long program_held_bytes(int *programs);

}  // namespace stl
