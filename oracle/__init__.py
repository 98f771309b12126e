"""FP64 CPU oracle for the coupled LB/bead-dynamics step.  Test infrastructure only."""
