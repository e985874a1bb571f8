"""qfuse: fused forward + adjoint-gradient simulation of batched parameterised circuits on MI355X."""
