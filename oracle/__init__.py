"""FP64 CPU oracle for the generalized Hermitian eigenproblem (test
infrastructure only; the product package never imports this)."""
