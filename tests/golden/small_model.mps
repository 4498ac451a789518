* A small LP written for the MPS reader tests (not from any library).
* maximise 3 x1 + 2 x2 - x3 + 4 x4 + 1.5
NAME          SMALLMODEL
OBJSENSE
    MAX
ROWS
 N  PROFIT
 L  CAP1
 G  DEMAND
 E  BAL
 L  RANGED
 N  FREEROW
COLUMNS
    X1        PROFIT         3.0   CAP1           1.0
    X1        BAL            1.0   FREEROW        9.0
    X2        PROFIT         2.0   CAP1           2.0
    X2        DEMAND         1.0   RANGED         1.0
    MARKER                 'MARKER'                 'INTORG'
    X3        PROFIT        -1.0   DEMAND         1.0
    X3        BAL           -1.0
    MARKER                 'MARKER'                 'INTEND'
    X4        PROFIT         4.0   CAP1           1.0
    X4        RANGED         2.0   RANGED         1.0
RHS
    RHS       PROFIT        -1.5   CAP1          10.0
    RHS       DEMAND         2.0   BAL            1.0
    RHS       RANGED         8.0
RANGES
    RNG       RANGED         5.0
BOUNDS
 UP BND       X1             4.0
 MI BND       X2
 UP BND       X2             6.0
 LO BND       X3            -2.0
 UP BND       X3             3.0
 UP BND       X4             2.5
ENDATA
