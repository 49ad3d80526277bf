"""MI355X (gfx950) library for the sparse robust l1 best-fit line of Ling &
Brooks, "l1-Norm Regularized l1-Norm Best-Fit Lines"."""
__all__ = ["binding", "workloads", "build"]
