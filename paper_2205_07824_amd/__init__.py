"""MI355X (gfx950) matrix-free LDG residual / Jacobian-vector product library with
Newton-GMRES solvers, block-Jacobi and learned element-patch preconditioners."""
