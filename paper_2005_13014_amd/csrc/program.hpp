// Batched timestep programs and reverse mode (program.cpp, adjoint.hip).
#pragma once

namespace stl {

// Releases cached graphs and tuned configurations of stencil_program_run.
void program_release_all();

}  // namespace stl
