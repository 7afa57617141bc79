"""FP64 CPU oracle for the adaptive mixed-precision H_h mat-vec (test
infrastructure only; see hh_oracle.py)."""
